"""MI355X (gfx950) COBS: compact bit-sliced signature index, query hot path.

Thin ctypes binding over ``libcobs.so`` (C ABI in ``include/cobs.h``).  This
layer only marshals arguments: every step of construction and query runs in
the library's HIP kernels.  PyTorch is used, when present, for device memory
(query bytes already resident in HBM) and for the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcobs.so")
_lib = None
_lock = threading.Lock()

OK, EINVAL, ENOMEM, EBUDGET, EOVERFLOW, EDEVICE, ECANCELLED, ESTATE = range(8)
DNA, BYTES = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
MODE_BATCHED, MODE_PLAIN = 0, 1
ORDER_AUTO, ORDER_QUERIES, ORDER_SLICES = 0, 1, 2   # cobs_order: gather work-item order
HOST_READS_AUTO, HOST_READS_STREAM, HOST_READS_IN_PLACE = 0, 1, 2   # cobs_host_reads
LAUNCH_AUTO, LAUNCH_DIRECT = 0, 1   # cobs_launch: replayed graphs for single short queries or not
PRUNE_OFF, PRUNE_ON = 0, 1          # cobs_prune: early exit of threshold queries (same results)


class CobsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cobs status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("q", C.c_uint32), ("canonical", C.c_uint32),
                ("num_hashes", C.c_uint32), ("fpr", C.c_double), ("block_docs", C.c_uint32),
                ("reserved", C.c_uint32), ("seed", C.c_uint64)]


class DocsC(C.Structure):
    _fields_ = [("bytes", C.c_void_p), ("str_off", C.c_void_p), ("doc_str", C.c_void_p),
                ("n_docs", C.c_uint32), ("mem", C.c_uint32)]


class IndexInfo(C.Structure):
    _fields_ = [("n_docs", C.c_uint32), ("n_blocks", C.c_uint32), ("params", Params),
                ("total_bytes", C.c_uint64), ("score_bytes", C.c_uint64),
                ("host_resident", C.c_uint32), ("n_groups", C.c_uint32),
                ("stage_bytes", C.c_uint64)]


class QueryOpts(C.Structure):
    _fields_ = [("k_num", C.c_uint32), ("k_den", C.c_uint32), ("topk", C.c_uint32),
                ("score_bits", C.c_uint32), ("mode", C.c_uint32), ("mem", C.c_uint32),
                ("chunk", C.c_uint32)]


class Hits(C.Structure):
    _fields_ = [("n", C.c_uint32), ("num_terms", C.c_uint32),
                ("doc_id", C.POINTER(C.c_uint32)), ("score", C.POINTER(C.c_uint32))]


class ServeOpts(C.Structure):
    _fields_ = [("score_budget_bytes", C.c_uint64), ("num_streams", C.c_uint32),
                ("max_batch_queries", C.c_uint32), ("max_batch_terms", C.c_uint64),
                ("score_bits", C.c_uint32), ("max_inflight", C.c_uint32)]


class ServeStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rejected", C.c_uint64),
                ("cancelled", C.c_uint64), ("batches", C.c_uint64), ("p50_ns", C.c_uint64),
                ("p99_ns", C.c_uint64), ("max_ns", C.c_uint64), ("queries_per_s", C.c_double),
                ("lookups_per_s", C.c_double), ("wall_s", C.c_double), ("lookups", C.c_uint64)]


class Tuning(C.Structure):
    _fields_ = [("unroll", C.c_uint32), ("chunk", C.c_uint32), ("gather_ms", C.c_double),
                ("order", C.c_uint32), ("host_reads", C.c_uint32), ("launch", C.c_uint32),
                ("prune", C.c_uint32)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_uint64)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class KernelTiming(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("total_ms", C.c_double), ("last_ms", C.c_double),
                ("row_bytes", C.c_uint64), ("terms", C.c_uint64)]


EXPORTS = {
    "cobs_build": (C.c_int, [C.POINTER(Params), C.POINTER(DocsC), C.c_void_p, C.POINTER(C.c_void_p)]),
    "cobs_builder_create": (C.c_int, [C.POINTER(Params), C.c_uint32, C.c_void_p,
                                      C.POINTER(C.c_void_p)]),
    "cobs_builder_count": (C.c_int, [C.c_void_p, C.POINTER(DocsC), C.c_uint32]),
    "cobs_builder_plan": (C.c_int, [C.c_void_p]),
    "cobs_builder_insert": (C.c_int, [C.c_void_p, C.POINTER(DocsC), C.c_uint32]),
    "cobs_builder_finish": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "cobs_builder_free": (None, [C.c_void_p]),
    "cobs_index_free": (None, [C.c_void_p]),
    "cobs_index_info": (C.c_int, [C.c_void_p, C.POINTER(IndexInfo)]),
    "cobs_index_block": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    "cobs_index_order": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "cobs_index_read": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p]),
    "cobs_index_merge": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "cobs_docset_create": (C.c_int, [C.POINTER(C.c_void_p)]),
    "cobs_docset_add_file": (C.c_int, [C.c_void_p, C.c_char_p, C.c_uint32]),
    "cobs_docset_add_buffer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32]),
    "cobs_docset_view": (C.c_int, [C.c_void_p, C.POINTER(DocsC)]),
    "cobs_docset_free": (None, [C.c_void_p]),
    "cobs_index_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "cobs_index_load": (C.c_int, [C.c_char_p, C.c_int, C.c_uint64, C.POINTER(C.c_void_p)]),
    "cobs_index_offload": (C.c_int, [C.c_void_p, C.c_uint64]),
    "cobs_index_onload": (C.c_int, [C.c_void_p]),
    "cobs_query_batch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                                   C.POINTER(QueryOpts), C.c_void_p, C.POINTER(C.POINTER(Hits))]),
    "cobs_query_scores": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "cobs_query_scores_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                                            C.c_void_p, C.c_void_p, C.c_void_p]),
    "cobs_query_terms": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "cobs_hits_free": (None, [C.POINTER(Hits), C.c_uint32]),
    "cobs_query_results": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                                     C.POINTER(QueryOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    "cobs_results_view": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32),
                                    C.POINTER(C.POINTER(C.c_uint32)),
                                    C.POINTER(C.POINTER(C.c_uint64)),
                                    C.POINTER(C.POINTER(C.c_uint32)),
                                    C.POINTER(C.POINTER(C.c_uint32))]),
    "cobs_results_free": (None, [C.c_void_p]),
    "cobs_set_allocator": (C.c_int, [C.POINTER(Allocator)]),
    "cobs_query_multi": (C.c_int, [C.POINTER(C.c_void_p), C.c_uint32, C.c_void_p, C.c_void_p,
                                   C.c_uint32, C.POINTER(QueryOpts), C.c_void_p,
                                   C.POINTER(C.c_void_p)]),
    "cobs_serve": (C.c_int, [C.c_void_p, C.POINTER(ServeOpts), C.POINTER(C.c_void_p)]),
    "cobs_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32,
                              C.c_uint32, C.c_uint64, C.POINTER(C.c_uint64)]),
    "cobs_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.POINTER(Hits)),
                            C.POINTER(C.c_uint64)]),
    "cobs_serve_stop": (C.c_int, [C.c_void_p, C.POINTER(ServeStats)]),
    "cobs_serve_replay": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                    C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p]),
    "cobs_tune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32,
                            C.c_void_p, C.POINTER(Tuning)]),
    "cobs_set_tuning": (C.c_int, [C.c_void_p, C.POINTER(Tuning)]),
    "cobs_profile": (C.c_int, [C.c_int]),
    "cobs_read_bandwidth": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p,
                                      C.POINTER(C.c_double)]),
    "cobs_read_rows_bandwidth": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint64, C.c_int,
                                           C.c_void_p, C.POINTER(C.c_double)]),
    "cobs_profile_read": (C.c_int, [C.POINTER(KernelTiming), C.c_int]),
    "cobs_last_error": (C.c_char_p, []),
    "cobs_now_ns": (C.c_uint64, []),
}


def lib():
    """Load libcobs.so (built in-tree by __graft_entry__.build()); fails loudly
    when it is missing -- there is no fallback path."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
            # torch first: the library then binds to the HIP runtime torch
            # loaded (same soname) instead of bringing a second one into the
            # process, which would not see the device
            import torch  # noqa: F401
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in EXPORTS.items():
                f = getattr(L, name)
                f.restype, f.argtypes = res, args
            _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise CobsError(status, lib().cobs_last_error().decode(errors="replace"))


def _p(a: np.ndarray):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _byte_source(data):
    """(pointer, mem, keepalive) for host numpy/bytes or a torch CUDA uint8 tensor."""
    if hasattr(data, "is_cuda") and data.is_cuda:
        return C.c_void_p(data.data_ptr()), MEM_DEVICE, data
    arr = np.frombuffer(data, np.uint8) if isinstance(data, (bytes, bytearray)) else \
        np.ascontiguousarray(data, dtype=np.uint8)
    if arr.size == 0:
        arr = np.zeros(1, np.uint8)
    return C.c_void_p(arr.ctypes.data), MEM_HOST, arr


def _docs_struct(data, str_off, doc_str):
    ptr, mem, keep = _byte_source(data)
    so = np.ascontiguousarray(str_off, dtype=np.uint64)
    ds = np.ascontiguousarray(doc_str, dtype=np.uint64)
    d = DocsC(ptr, C.c_void_p(so.ctypes.data), C.c_void_p(ds.ctypes.data), len(ds) - 1, mem)
    return d, (keep, so, ds)


FASTA, MULTI_FASTA, FASTQ, TEXT = range(4)


class DocSet:
    """Documents read from FASTA / multi-FASTA / FASTQ / text files or buffers
    (cobs_docset_*); arrays() gives (bytes, str_off, doc_str) for Index.build
    or as queries."""

    def __init__(self):
        self._h = C.c_void_p()
        _check(lib().cobs_docset_create(C.byref(self._h)))

    def __del__(self):
        if getattr(self, "_h", None):
            lib().cobs_docset_free(self._h)
            self._h = None

    def add_file(self, path: str, fmt: int) -> "DocSet":
        _check(lib().cobs_docset_add_file(self._h, os.fsencode(path), fmt))
        return self

    def add_buffer(self, data: bytes, fmt: int) -> "DocSet":
        buf = np.frombuffer(data, np.uint8) if len(data) else np.zeros(1, np.uint8)
        _check(lib().cobs_docset_add_buffer(self._h, C.c_void_p(buf.ctypes.data), len(data), fmt))
        return self

    def arrays(self):
        d = DocsC()
        _check(lib().cobs_docset_view(self._h, C.byref(d)))
        n_str = 0
        ds = np.ctypeslib.as_array(C.cast(d.doc_str, C.POINTER(C.c_uint64)), (d.n_docs + 1,)).copy()
        n_str = int(ds[-1])
        so = np.ctypeslib.as_array(C.cast(d.str_off, C.POINTER(C.c_uint64)), (n_str + 1,)).copy()
        nb = int(so[-1])
        data = (np.ctypeslib.as_array(C.cast(d.bytes, C.POINTER(C.c_uint8)), (nb,)).copy()
                if nb else np.zeros(0, np.uint8))
        return data, so, ds


def make_params(kind=DNA, q=31, canonical=True, h=1, p=0.3, B=0, seed=0x5EED) -> Params:
    return Params(kind, q, int(canonical), h, p, B, 0, seed)


class Index:
    """A COBS index: the matrix in HBM of its device, or in pinned host memory
    after offload (streamed per query batch)."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def build(cls, params: Params, data, str_off, doc_str, stream=None) -> "Index":
        d, keep = _docs_struct(data, str_off, doc_str)
        h = C.c_void_p()
        _check(lib().cobs_build(C.byref(params), C.byref(d), _stream(stream), C.byref(h)))
        return cls(h)

    @classmethod
    def load(cls, path: str, device: int = 0, device_budget_bytes: int = 0) -> "Index":
        """Index from a file written by save (cobs_index_load); a non-zero
        budget keeps the matrix in host memory, streamed per batch."""
        h = C.c_void_p()
        _check(lib().cobs_index_load(os.fsencode(path), device, device_budget_bytes, C.byref(h)))
        return cls(h)

    def merge(self, other: "Index") -> "Index":
        """A new index: this one's documents, then other's (cobs_index_merge)."""
        h = C.c_void_p()
        _check(lib().cobs_index_merge(self._h, other._h, C.byref(h)))
        return Index(h)

    def save(self, path: str) -> None:
        """Write the index to a file (cobs_index_save)."""
        _check(lib().cobs_index_save(self._h, os.fsencode(path)))

    @classmethod
    def build_streamed(cls, params: Params, n_docs: int, runs, stream=None) -> "Index":
        """runs(pass_no) yields (first, data, str_off, doc_str) for every run of
        documents; it is called once for the counting pass and once for the
        insertion pass."""
        b = C.c_void_p()
        st = _stream(stream)
        _check(lib().cobs_builder_create(C.byref(params), n_docs, st, C.byref(b)))
        try:
            for first, data, so, ds in runs(0):
                d, keep = _docs_struct(data, so, ds)
                _check(lib().cobs_builder_count(b, C.byref(d), first))
            _check(lib().cobs_builder_plan(b))
            for first, data, so, ds in runs(1):
                d, keep = _docs_struct(data, so, ds)
                _check(lib().cobs_builder_insert(b, C.byref(d), first))
            h = C.c_void_p()
            _check(lib().cobs_builder_finish(b, C.byref(h)))
            return cls(h)
        finally:
            lib().cobs_builder_free(b)

    def close(self):
        if self._h:
            lib().cobs_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = IndexInfo()
        _check(lib().cobs_index_info(self._h, C.byref(i)))
        return dict(n_docs=i.n_docs, n_blocks=i.n_blocks, total_bytes=i.total_bytes,
                    score_bytes=i.score_bytes, host_resident=bool(i.host_resident),
                    n_groups=i.n_groups, stage_bytes=i.stage_bytes)

    def offload(self, device_budget_bytes: int) -> None:
        """Matrix to pinned host memory; queries stream it (cobs_index_offload)."""
        _check(lib().cobs_index_offload(self._h, device_budget_bytes))

    def onload(self) -> None:
        """Matrix back into device memory (cobs_index_onload)."""
        _check(lib().cobs_index_onload(self._h))

    def block(self, b: int) -> dict:
        f, d = C.c_uint32(), C.c_uint32()
        r, s, o = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(lib().cobs_index_block(self._h, b, C.byref(f), C.byref(d), C.byref(r),
                                      C.byref(s), C.byref(o)))
        return dict(first=f.value, docs=d.value, rows=r.value, stride=s.value, offset=o.value)

    def order(self):
        n = self.info()["n_docs"]
        order = np.zeros(max(n, 1), np.uint32)
        nt = np.zeros(max(n, 1), np.uint64)
        _check(lib().cobs_index_order(self._h, _p(order), _p(nt)))
        return order[:n], nt[:n]

    def read(self, offset: int, nbytes: int) -> np.ndarray:
        out = np.zeros(max(nbytes, 1), np.uint8)
        _check(lib().cobs_index_read(self._h, offset, nbytes, _p(out)))
        return out[:nbytes]

    def tune(self, data, q_off, stream=None) -> dict:
        """Autotune the gather launch shape on a sample batch (kept by the index)."""
        ptr, mem, keep = _byte_source(data)
        qo = np.ascontiguousarray(q_off, dtype=np.uint64)
        t = Tuning()
        _check(lib().cobs_tune(self._h, ptr, _p(qo), len(qo) - 1, mem, _stream(stream),
                               C.byref(t)))
        return dict(unroll=t.unroll, chunk=t.chunk, order=t.order, gather_ms=t.gather_ms)

    def set_tuning(self, unroll=0, chunk=0, order=ORDER_AUTO, host_reads=HOST_READS_AUTO,
                   launch=LAUNCH_AUTO, prune=PRUNE_OFF) -> None:
        """cobs_set_tuning: every field at once (0 = default); results never
        depend on any of them."""
        t = Tuning(unroll, chunk, 0.0, order, host_reads, launch, prune)
        _check(lib().cobs_set_tuning(self._h, C.byref(t)))

    def query_flat(self, data, q_off, k=(4, 5), topk=0, score_bits=32, mode=MODE_BATCHED,
                   stream=None, chunk=0):
        """Hits of every query in flat arrays: (num_terms[n], hit_off[n+1],
        doc_ids[total], scores[total]); query i's hits are
        doc_ids[hit_off[i]:hit_off[i+1]]."""
        ptr, mem, keep = _byte_source(data)
        qo = np.ascontiguousarray(q_off, dtype=np.uint64)
        n = len(qo) - 1
        opts = QueryOpts(k[0], k[1], topk, score_bits, mode, mem, chunk)
        r = C.c_void_p()
        _check(lib().cobs_query_results(self._h, ptr, _p(qo), n, C.byref(opts), _stream(stream),
                                        C.byref(r)))
        return _take_results(r, n)

    def query(self, data, q_off, k=(4, 5), topk=0, score_bits=32, mode=MODE_BATCHED,
              stream=None, chunk=0):
        """Hits of every query: list of (doc_ids, scores, num_terms)."""
        nt, off, ids, sc = self.query_flat(data, q_off, k, topk, score_bits, mode, stream, chunk)
        return [(ids[off[i]:off[i + 1]], sc[off[i]:off[i + 1]], int(nt[i]))
                for i in range(len(nt))]

    def query_hits(self, data, q_off, k=(4, 5), topk=0, score_bits=32, mode=MODE_BATCHED,
                   stream=None, chunk=0):
        """The same through cobs_query_batch (one cobs_hits per query)."""
        ptr, mem, keep = _byte_source(data)
        qo = np.ascontiguousarray(q_off, dtype=np.uint64)
        n = len(qo) - 1
        opts = QueryOpts(k[0], k[1], topk, score_bits, mode, mem, chunk)
        out = C.POINTER(Hits)()
        _check(lib().cobs_query_batch(self._h, ptr, _p(qo), n, C.byref(opts), _stream(stream),
                                      C.byref(out)))
        try:
            res = []
            for i in range(n):
                h = out[i]
                ids = np.ctypeslib.as_array(h.doc_id, (max(h.n, 1),))[: h.n].copy()
                sc = np.ctypeslib.as_array(h.score, (max(h.n, 1),))[: h.n].copy()
                res.append((ids, sc, int(h.num_terms)))
            return res
        finally:
            lib().cobs_hits_free(out, n)

    def scores(self, data, q_off, stream=None):
        """Full score matrix [n_queries, n_docs] (input ids) and l per query."""
        ptr, mem, keep = _byte_source(data)
        qo = np.ascontiguousarray(q_off, dtype=np.uint64)
        n = len(qo) - 1
        nd = self.info()["n_docs"]
        sc = np.zeros((max(n, 1), max(nd, 1)), np.uint32)
        nt = np.zeros(max(n, 1), np.uint32)
        _check(lib().cobs_query_scores(self._h, ptr, _p(qo), n, mem, _stream(stream), _p(sc), _p(nt)))
        return sc[:n, :nd], nt[:n]

    def scores_noalloc(self, data, q_off, scores, num_terms=None, stream=None):
        """Full scores into caller-owned device tensors without any device
        allocation (cobs_query_scores_noalloc): data is a device uint8 tensor,
        scores a device int32/uint32 tensor of n_queries * n_docs elements,
        num_terms one of n_queries elements or None.  Asynchronous on the
        stream (torch's current one by default)."""
        qo = np.ascontiguousarray(q_off, dtype=np.uint64)
        n = len(qo) - 1
        nd = self.info()["n_docs"]
        if not data.is_cuda or not scores.is_cuda or (num_terms is not None and not num_terms.is_cuda):
            raise ValueError("data, scores and num_terms must be device tensors")
        if scores.numel() * scores.element_size() < n * nd * 4:
            raise ValueError("scores holds fewer than n_queries * n_docs 32-bit words")
        if num_terms is not None and num_terms.numel() * num_terms.element_size() < n * 4:
            raise ValueError("num_terms holds fewer than n_queries 32-bit words")
        _check(lib().cobs_query_scores_noalloc(
            self._h, C.c_void_p(data.data_ptr()), _p(qo), n, _stream(stream),
            C.c_void_p(scores.data_ptr()),
            C.c_void_p(num_terms.data_ptr()) if num_terms is not None else None))

    def terms(self, data, q_off, q: int, stream=None):
        """Distinct terms of each query (unordered within a query)."""
        ptr, mem, keep = _byte_source(data)
        qo = np.ascontiguousarray(q_off, dtype=np.uint64)
        n = len(qo) - 1
        lens = np.diff(qo.astype(np.int64))
        nw = np.maximum(lens - q + 1, 0)
        base = np.concatenate([[0], np.cumsum(nw)]).astype(np.int64)
        t = np.zeros(max(int(base[-1]), 1), np.uint64)
        nt = np.zeros(max(n, 1), np.uint32)
        _check(lib().cobs_query_terms(self._h, ptr, _p(qo), n, mem, _stream(stream), _p(t), _p(nt)))
        return [t[base[i]:base[i] + nt[i]].copy() for i in range(n)]


class Server:
    """Continuous-batching server over a resident index (cobs_serve)."""

    def __init__(self, index: Index, budget_bytes=0, num_streams=0, max_batch_queries=0,
                 max_batch_terms=0, score_bits=32, max_inflight=0):
        self.index = index
        opts = ServeOpts(budget_bytes, num_streams, max_batch_queries, max_batch_terms,
                         score_bits, max_inflight)
        self._h = C.c_void_p()
        _check(lib().cobs_serve(index._h, C.byref(opts), C.byref(self._h)))

    def submit(self, query: bytes, k=(4, 5), topk=0, arrival_ns=0) -> int:
        arr = np.frombuffer(query, np.uint8) if len(query) else np.zeros(1, np.uint8)
        t = C.c_uint64()
        _check(lib().cobs_submit(self._h, C.c_void_p(arr.ctypes.data), len(query), k[0], k[1],
                                 topk, arrival_ns, C.byref(t)))
        return t.value

    def wait(self, ticket: int):
        out = C.POINTER(Hits)()
        lat = C.c_uint64()
        _check(lib().cobs_wait(self._h, ticket, C.byref(out), C.byref(lat)))
        try:
            h = out[0]
            ids = np.ctypeslib.as_array(h.doc_id, (max(h.n, 1),))[: h.n].copy()
            sc = np.ctypeslib.as_array(h.score, (max(h.n, 1),))[: h.n].copy()
            return ids, sc, int(h.num_terms), lat.value
        finally:
            lib().cobs_hits_free(out, 1)

    def replay(self, data, q_off, arrival_s, k=(4, 5), topk=0):
        """Open-loop replay: query i submitted at its scheduled arrival (seconds
        from now) by a native thread; returns (latency_ns, n_hits) arrays."""
        arr = np.ascontiguousarray(data, dtype=np.uint8)
        if arr.size == 0:
            arr = np.zeros(1, np.uint8)
        qo = np.ascontiguousarray(q_off, dtype=np.uint64)
        n = len(qo) - 1
        at = np.ascontiguousarray(np.round(np.asarray(arrival_s) * 1e9), dtype=np.uint64)
        lat = np.zeros(max(n, 1), np.uint64)
        nh = np.zeros(max(n, 1), np.uint32)
        _check(lib().cobs_serve_replay(self._h, C.c_void_p(arr.ctypes.data), _p(qo), n, _p(at),
                                       k[0], k[1], topk, _p(lat), _p(nh)))
        return lat[:n], nh[:n]

    def stop(self) -> dict:
        st = ServeStats()
        _check(lib().cobs_serve_stop(self._h, C.byref(st)))
        self._h = None
        return {f: getattr(st, f) for f, _ in ServeStats._fields_}


def _take_results(r, n):
    """Copy a cobs_results object into numpy arrays and free it."""
    try:
        nq = C.c_uint32()
        nt, off, ids, sc = (C.POINTER(C.c_uint32)(), C.POINTER(C.c_uint64)(),
                            C.POINTER(C.c_uint32)(), C.POINTER(C.c_uint32)())
        _check(lib().cobs_results_view(r, C.byref(nq), C.byref(nt), C.byref(off),
                                       C.byref(ids), C.byref(sc)))
        num_terms = np.ctypeslib.as_array(nt, (n,)).copy() if n else np.zeros(0, np.uint32)
        hit_off = np.ctypeslib.as_array(off, (n + 1,)).copy()
        total = int(hit_off[-1])
        if total:
            doc_ids = np.ctypeslib.as_array(ids, (total,)).copy()
            scores = np.ctypeslib.as_array(sc, (total,)).copy()
        else:
            doc_ids = np.zeros(0, np.uint32)
            scores = np.zeros(0, np.uint32)
        return num_terms, hit_off, doc_ids, scores
    finally:
        lib().cobs_results_free(r)


def query_multi(indexes, data, q_off, k=(4, 5), topk=0, score_bits=32, mode=MODE_BATCHED,
                stream=None, chunk=0):
    """Query several indexes as one collection (cobs_query_multi): list of
    (doc_ids, scores, num_terms) per query, ids numbered across the indexes
    in order."""
    ptr, mem, keep = _byte_source(data)
    qo = np.ascontiguousarray(q_off, dtype=np.uint64)
    n = len(qo) - 1
    opts = QueryOpts(k[0], k[1], topk, score_bits, mode, mem, chunk)
    hs = (C.c_void_p * max(len(indexes), 1))(*[ix._h for ix in indexes])
    r = C.c_void_p()
    _check(lib().cobs_query_multi(hs, len(indexes), ptr, _p(qo), n, C.byref(opts),
                                  _stream(stream), C.byref(r)))
    nt, off, ids, sc = _take_results(r, n)
    return [(ids[off[i]:off[i + 1]], sc[off[i]:off[i + 1]], int(nt[i])) for i in range(n)]


# every allocator pair ever installed: memory it handed out is given back
# through it, possibly long after another pair replaced it
_ALLOCATORS = []


def set_allocator(alloc=None, free=None) -> None:
    """Route the library's device allocations through alloc(bytes) -> int
    pointer (0 on failure) and free(pointer) (cobs_set_allocator); with no
    arguments, back to hipMalloc/hipFree."""
    if alloc is None:
        _check(lib().cobs_set_allocator(None))
        return

    def _a(ctx, n):
        try:
            return int(alloc(int(n))) or None
        except Exception:
            return None

    def _f(ctx, ptr):
        free(int(ptr))

    pair = Allocator(_ALLOC_FN(_a), _FREE_FN(_f), None)
    _ALLOCATORS.append(pair)
    _check(lib().cobs_set_allocator(C.byref(pair)))


def use_torch_allocator(enable: bool = True) -> None:
    """Take the library's device memory from torch's caching allocator (so
    that torch and the library share one pool), or give that up."""
    if not enable:
        set_allocator()
        return
    import torch
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n),
                  lambda ptr: torch.cuda.caching_allocator_delete(ptr))


def now_ns() -> int:
    return int(lib().cobs_now_ns())


def read_bandwidth(tensor, stream=None) -> float:
    """GB/s of one coalesced read pass over a device tensor (cobs_read_bandwidth)."""
    gbps = C.c_double()
    nbytes = tensor.numel() * tensor.element_size() // 16 * 16
    _check(lib().cobs_read_bandwidth(C.c_void_p(tensor.data_ptr()), nbytes, _stream(stream),
                                     C.byref(gbps)))
    return gbps.value


def read_rows_bandwidth(tensor, reads: int, cached: bool = True, stream=None) -> float:
    """GB/s of random 1 KiB row reads over a device tensor
    (cobs_read_rows_bandwidth): cached loads over a buffer that fits in the
    caches measure the cache-resident ceiling."""
    gbps = C.c_double()
    nbytes = tensor.numel() * tensor.element_size()
    _check(lib().cobs_read_rows_bandwidth(C.c_void_p(tensor.data_ptr()), nbytes, int(reads),
                                          1 if cached else 0, _stream(stream), C.byref(gbps)))
    return gbps.value


def profile(enable: bool) -> None:
    """Time every gather-kernel launch with HIP events on its own stream."""
    _check(lib().cobs_profile(1 if enable else 0))


def profile_read(reset: bool = False) -> dict:
    t = KernelTiming()
    _check(lib().cobs_profile_read(C.byref(t), 1 if reset else 0))
    return {f: getattr(t, f) for f, _ in KernelTiming._fields_}
