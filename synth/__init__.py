"""Seeded synthetic inputs shaped like the COBS workloads.

The paper evaluates on 100,000 de-noised microbial McCortex k-mer files
(section 3), which are not available here; these generators stand in for
them with random ACGT documents whose distinct 31-mer counts follow the
stated size distributions, Zipf text documents, and query sets of planted
substrings (with substitutions) and random strings.

The module holds none of the index or query arithmetic: it only produces
bytes.  Every random number is a Philox4x32-10 output addressed by
(index, sub-index, stream) under the config's 64-bit seed (synth.c), so the
same document can be regenerated on the host or, for the large workloads, on
the device (synth_dev.hip) bit-identically.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field, replace

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_DIR, "libsynth.so")
_DEVLIB = os.path.join(_DIR, "libsynth_dev.so")
_lib = None
_devlib = None
_lock = threading.Lock()

HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(device: bool = True) -> None:
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           os.path.join(_DIR, "synth.c"), "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    if device:
        tmp = _DEVLIB + ".tmp"
        subprocess.check_call(["/opt/rocm/bin/hipcc", *HIP_FLAGS,
                               os.path.join(_DIR, "synth_dev.hip"), "-o", tmp])
        os.replace(tmp, _DEVLIB)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(device=False)
            L = C.CDLL(_LIB)
            u64, u32, vp, dbl = C.c_uint64, C.c_uint32, C.c_void_p, C.c_double
            sig = {
                "synth_philox": (None, [vp, vp, vp]),
                "synth_doc_bases": (None, [u64, u32, u64, u64, vp]),
                "synth_doc_lengths": (None, [u64, C.c_int, u32, dbl, dbl, dbl, dbl, u32, vp]),
                "synth_dna_query": (u64, [u64, u32, C.c_int, dbl, dbl, C.c_int, dbl, u32,
                                          vp, vp, vp, vp]),
                "synth_word": (u32, [u64, u32, u32, u32, vp]),
                "synth_zipf_cdf": (None, [u32, dbl, vp]),
                "synth_text_doc": (None, [u64, u32, u64, vp, u32, vp, vp, u32, vp]),
                "synth_text_lengths": (None, [u64, u32, dbl, dbl, dbl, dbl, vp]),
                "synth_text_query": (u64, [u64, u32, u64, u64, dbl, u32, vp, vp, vp, vp]),
                "synth_arrivals": (None, [u64, u32, dbl, u32, vp]),
                "synth_uniform": (dbl, [u64, u32, u64, u32]),
                "synth_doc_base": (C.c_uint8, [u64, u32, u64]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype, f.argtypes = res, args
            _lib = L
    return _lib


def devlib():
    """Device generator (HIP); only for GPU runs."""
    global _devlib
    with _lock:
        if _devlib is None:
            if not os.path.exists(_DEVLIB):
                raise RuntimeError("synth/libsynth_dev.so is not built "
                                   "(run __graft_entry__.build())")
            import torch  # noqa: F401  (bind to torch's HIP runtime, not a second copy)
            L = C.CDLL(_DEVLIB)
            L.synth_dev_doc_bases.restype = C.c_int
            L.synth_dev_doc_bases.argtypes = [C.c_uint64, C.c_void_p, C.c_uint32,
                                              C.c_uint32, C.c_void_p, C.c_void_p]
            _devlib = L
    return _devlib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    c = np.array(ctr, np.uint32)
    k = np.array(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().synth_philox(_p(c), _p(k), _p(o))
    return [int(x) for x in o]


# ---- workload descriptions --------------------------------------------------

@dataclass
class Workload:
    name: str
    kind: str                      # "dna" | "text"
    n_docs: int
    doc_size: tuple                # see synth_doc_lengths / text lengths
    q: int
    canonical: bool
    h: int
    p: float
    B: int                         # 0 = classic
    n_queries: int
    q_len: tuple                   # ("fixed", L) | ("loguniform", a, b) | ("uniform", a, b)
    planted_every: int = 2
    subst: float = 0.01
    k: tuple = (4, 5)
    topk: int = 0
    score_bits: int = 32
    seed: int = 0
    hash_seed: int = 0x5EED
    vocab: int = 50_000
    zipf: float = 1.1
    word_len: tuple = (4, 12)
    extra: dict = field(default_factory=dict)

    def scaled(self, s: int, name: str | None = None) -> "Workload":
        """A smaller copy: documents, sizes, block size and query count
        divided by s (query lengths kept unless they exceed the documents)."""
        ds = self.doc_size
        if ds[0] in ("uniform", "target_uniform"):
            ds = (ds[0], max(ds[1] // s, 40), max(ds[2] // s, 41))
        elif ds[0] == "lognormal":
            ds = (ds[0], ds[1] / s, ds[2], ds[3] / s)
        elif ds[0] == "text_lognormal":
            ds = (ds[0], ds[1] / s, ds[2], ds[3] / s)
        return replace(self, name=name or f"{self.name}/s{s}",
                       n_docs=max(self.n_docs // s, 2), doc_size=ds,
                       B=(max(self.B // s, 8) if self.B else 0),
                       n_queries=max(self.n_queries // s, 4))


CONFIGS = {
    1: Workload("classic-1k", "dna", 1000, ("uniform", 10_000, 100_000), 31, True, 1, 0.3,
                0, 100, ("fixed", 1000), score_bits=16, seed=0xC0B50001),
    2: Workload("classic-10k", "dna", 10_000, ("target_uniform", 100_000, 1_000_000), 31,
                True, 1, 0.3, 0, 10_000, ("loguniform", 100, 10_000), seed=0xC0B50002),
    3: Workload("compact-100k", "dna", 100_000, ("lognormal", 1e6, 0.7, 8e6), 31, True, 1,
                0.3, 8192, 10_000, ("loguniform", 100, 10_000), topk=100, seed=0xC0B50003),
    4: Workload("text-50k", "text", 50_000, ("text_lognormal", 20_000, 0.7, 320_000), 8,
                False, 3, 0.1, 8192, 65_536, ("uniform", 16, 4096), seed=0xC0B50004),
    5: Workload("serve-100k", "dna", 100_000, ("lognormal", 1e6, 0.7, 8e6), 31, True, 1,
                0.3, 8192, 20_000, ("loguniform", 31, 1_000_000), seed=0xC0B50003,
                extra={"rates": [1000, 2700, 7100, 18800, 50000]}),
}


# ---- documents --------------------------------------------------------------

def doc_lengths(w: Workload) -> np.ndarray:
    n = w.n_docs
    out = np.zeros(max(n, 1), np.uint64)
    ds = w.doc_size
    if ds[0] == "uniform":
        lib().synth_doc_lengths(w.seed, 0, n, ds[1], ds[2], 0.0, 0.0, w.q, _p(out))
    elif ds[0] == "target_uniform":
        lib().synth_doc_lengths(w.seed, 1, n, ds[1], ds[2], 0.0, 0.0, w.q, _p(out))
    elif ds[0] == "lognormal":
        lib().synth_doc_lengths(w.seed, 2, n, ds[1], 0.0, ds[2], ds[3], w.q, _p(out))
    elif ds[0] == "text_lognormal":
        lib().synth_text_lengths(w.seed, n, ds[1], ds[2], 1.0, ds[3], _p(out))
    else:
        raise ValueError(ds)
    return out[:n]


@dataclass
class DocSet:
    """Documents in CSR form (one string per document here)."""
    bytes: np.ndarray
    str_off: np.ndarray
    doc_str: np.ndarray

    @property
    def n_docs(self) -> int:
        return len(self.doc_str) - 1


def _csr(lengths: np.ndarray):
    off = np.zeros(len(lengths) + 1, np.uint64)
    np.cumsum(lengths, out=off[1:])
    return off, np.arange(len(lengths) + 1, dtype=np.uint64)


def dna_docs(w: Workload, first: int = 0, count: int | None = None,
             threads: int = 8) -> DocSet:
    """Host bytes of documents [first, first+count)."""
    lens = doc_lengths(w)
    count = w.n_docs - first if count is None else count
    sel = lens[first:first + count]
    str_off, doc_str = _csr(sel)
    data = np.empty(int(str_off[-1]) if count else 0, np.uint8)
    L = lib()

    def one(i):
        n = int(sel[i])
        if n:
            view = data[int(str_off[i]):int(str_off[i]) + n]
            L.synth_doc_bases(w.seed, first + i, 0, n, _p(view))

    if count:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(count)))
    return DocSet(data, str_off, doc_str)


def dna_docs_device(w: Workload, first: int, count: int, dev_bytes_ptr: int,
                    dev_off_ptr: int, stream_ptr: int = 0) -> None:
    """Generate documents [first, first+count) straight into device memory:
    dev_off_ptr points to count+1 device uint64 offsets (relative to
    dev_bytes_ptr)."""
    rc = devlib().synth_dev_doc_bases(w.seed, C.c_void_p(dev_off_ptr), first, count,
                                      C.c_void_p(dev_bytes_ptr), C.c_void_p(stream_ptr))
    if rc != 0:
        raise RuntimeError(f"synth_dev_doc_bases failed ({rc})")


class Vocab:
    def __init__(self, w: Workload):
        self.V = w.vocab
        self.wmax = w.word_len[1]
        self.words = np.zeros(self.V * self.wmax, np.uint8)
        self.wlen = np.zeros(self.V, np.uint32)
        for i in range(self.V):
            self.wlen[i] = lib().synth_word(w.seed, i, w.word_len[0], w.word_len[1],
                                            _p(self.words[i * self.wmax:]))
        self.cdf = np.zeros(self.V, np.float64)
        lib().synth_zipf_cdf(self.V, w.zipf, _p(self.cdf))


def text_docs(w: Workload, threads: int = 8) -> DocSet:
    lens = doc_lengths(w)
    str_off, doc_str = _csr(lens)
    data = np.empty(int(str_off[-1]), np.uint8)
    voc = Vocab(w)
    L = lib()

    def one(d):
        n = int(lens[d])
        view = data[int(str_off[d]):int(str_off[d]) + n]
        L.synth_text_doc(w.seed, d, n, _p(voc.cdf), voc.V, _p(voc.words), _p(voc.wlen),
                         voc.wmax, _p(view))

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, range(w.n_docs)))
    return DocSet(data, str_off, doc_str)


def docs(w: Workload) -> DocSet:
    return dna_docs(w) if w.kind == "dna" else text_docs(w)


# ---- queries ----------------------------------------------------------------

@dataclass
class QuerySet:
    bytes: np.ndarray
    q_off: np.ndarray
    src: np.ndarray                # source document of planted queries, -1 if random

    @property
    def n(self) -> int:
        return len(self.q_off) - 1

    def get(self, i: int) -> bytes:
        return self.bytes[int(self.q_off[i]):int(self.q_off[i + 1])].tobytes()

    def subset(self, idx) -> "QuerySet":
        parts = [self.bytes[int(self.q_off[i]):int(self.q_off[i + 1])] for i in idx]
        lens = np.array([len(p) for p in parts], np.uint64)
        off = np.zeros(len(parts) + 1, np.uint64)
        np.cumsum(lens, out=off[1:])
        data = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        return QuerySet(data, off, self.src[list(idx)])


def dna_queries(w: Workload, n: int | None = None, first: int = 0,
                doc_len: np.ndarray | None = None) -> QuerySet:
    n = w.n_queries if n is None else n
    lens_docs = doc_lengths(w) if doc_len is None else doc_len
    ql = w.q_len
    if ql[0] == "fixed":
        kind, a, b = 0, float(ql[1]), float(ql[1])
    elif ql[0] == "loguniform":
        kind, a, b = 1, float(ql[1]), float(ql[2])
    else:
        raise ValueError(ql)
    L = lib()
    lens = np.zeros(n, np.uint64)
    for i in range(n):
        lens[i] = L.synth_dna_query(w.seed, first + i, kind, a, b, w.planted_every, w.subst,
                                    w.n_docs, _p(lens_docs), None, None, None)
    off = np.zeros(n + 1, np.uint64)
    np.cumsum(lens, out=off[1:])
    data = np.empty(int(off[-1]), np.uint8)
    src = np.zeros(n, np.int64)
    s = C.c_int64()
    o = C.c_uint64()
    for i in range(n):
        view = data[int(off[i]):]
        L.synth_dna_query(w.seed, first + i, kind, a, b, w.planted_every, w.subst,
                          w.n_docs, _p(lens_docs), _p(view) if lens[i] else None,
                          C.byref(s), C.byref(o))
        src[i] = s.value
    return QuerySet(data, off, src)


def text_queries(w: Workload, d: DocSet, n: int | None = None) -> QuerySet:
    n = w.n_queries if n is None else n
    a, b = w.q_len[1], w.q_len[2]
    L = lib()
    lens = np.zeros(n, np.uint64)
    for i in range(n):
        lens[i] = L.synth_text_query(w.seed, i, a, b, w.subst, d.n_docs, _p(d.str_off),
                                     _p(d.bytes), None, None)
    off = np.zeros(n + 1, np.uint64)
    np.cumsum(lens, out=off[1:])
    data = np.empty(int(off[-1]), np.uint8)
    src = np.zeros(n, np.int64)
    s = C.c_int64()
    for i in range(n):
        L.synth_text_query(w.seed, i, a, b, w.subst, d.n_docs, _p(d.str_off), _p(d.bytes),
                           _p(data[int(off[i]):]), C.byref(s))
        src[i] = s.value
    return QuerySet(data, off, src)


def arrivals(seed: int, n: int, rate: float, tag: int = 0) -> np.ndarray:
    t = np.zeros(n, np.float64)
    lib().synth_arrivals(seed, n, rate, tag, _p(t))
    return t


def doc_base(seed: int, d: int, i: int) -> int:
    return int(lib().synth_doc_base(seed, d, i))


def uniform(seed: int, stream: int, idx: int, sub: int) -> float:
    return float(lib().synth_uniform(seed, stream, idx, sub))
