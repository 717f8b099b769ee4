"""Plain CPU oracle of the COBS query path (ctypes wrapper over cobs_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use this package; the product
library never does.  It shares no code with the GPU path.

What each function follows in the paper (Bingmann et al., COBS, 2019):

* ``terms`` / ``unique``          -- q-grams of a string and the set G_q
                                      (section 2.1), canonical k-mers
                                      (section 2.3)
* ``filter_rows``                 -- Bloom filter size from the false-positive
                                      formula of section 2.1 with h fixed
* ``bloom_fpr`` / ``binom_tail_gt`` / ``chernoff`` -- closed forms of section
                                      2.1 (Bloom FPR, Theorem 1, Chernoff)
* ``OracleIndex``                 -- classic / compact bit-sliced matrix
                                      (sections 2.2, 2.3) and the
                                      hash-AND-ADD-threshold query (section 2.2)
* ``bruteforce_scores``           -- the query score written without a matrix
* ``exact_intersection``          -- |G(P) cap G(d)|, the no-false-negative
                                      lower bound (sections 2.1, 2.2)

Parity unpinned by the paper: hash values, bit positions and exact score
integers (the paper prints none); they are pinned by brute force, invariants
and closed forms in the tests.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_DIR, "liboracle.so")
_lib = None
_lock = threading.Lock()

DNA, BYTES = 0, 1


def build() -> str:
    """Compile the oracle with gcc (plain C11, -O2)."""
    src = os.path.join(_DIR, "cobs_oracle.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", src,
                           "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("kind", C.c_int), ("q", C.c_uint32), ("canonical", C.c_int),
                ("h", C.c_uint32), ("p", C.c_double), ("B", C.c_uint32),
                ("seed", C.c_uint64), ("row_align", C.c_uint32)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build()
            L = C.CDLL(_LIB_PATH)
            u64, u32, vp = C.c_uint64, C.c_uint32, C.c_void_p
            sig = {
                "orc_splitmix64_next": (u64, [C.POINTER(u64)]),
                "orc_mix64": (u64, [u64]),
                "orc_term_hash": (u64, [u64, u64, u32]),
                "orc_terms": (u64, [C.c_int, u32, C.c_int, vp, u64, vp]),
                "orc_unique": (u64, [vp, u64]),
                "orc_filter_rows": (u64, [u64, u32, C.c_double]),
                "orc_bloom_fpr": (C.c_double, [C.c_double, u32, C.c_double]),
                "orc_bloom_fpr_exp": (C.c_double, [C.c_double, u32, C.c_double]),
                "orc_binom_tail_gt": (C.c_double, [u64, C.c_double, u64]),
                "orc_chernoff": (C.c_double, [u64, C.c_double, C.c_double]),
                "orc_build": (vp, [C.POINTER(_Params), vp, vp, vp, u32]),
                "orc_plan": (u32, [vp, u32, u32, vp, vp, vp, vp]),
                "orc_free": (None, [vp]),
                "orc_bit": (C.c_int, [vp, u32, u64, u32]),
                "orc_query_scores": (u64, [vp, vp, u64, vp]),
                "orc_report": (u32, [vp, u32, u64, u32, u32, u32, vp, vp]),
                "orc_bruteforce_scores": (u64, [C.POINTER(_Params), vp, vp, vp, u32,
                                                vp, u64, vp]),
                "orc_exact_intersection": (u64, [C.POINTER(_Params), vp, vp, vp, u32,
                                                 vp, u64, vp]),
                "orc_term_rows": (None, [C.POINTER(_Params), u64, vp, u64, vp]),
                "orc_doc_scores": (None, [C.POINTER(_Params), u64, vp, vp, u64, vp, u64, vp, u32,
                                          vp]),
                "orc_rc_palindrome_dups": (u64, [u32, vp, u64, C.POINTER(u64)]),
                "orc_n_blocks": (u32, [vp]),
                "orc_block_info": (None, [vp, u32, vp, vp, vp, vp, vp]),
                "orc_order": (vp, [vp]),
                "orc_n_terms": (vp, [vp]),
                "orc_bits": (vp, [vp]),
                "orc_total_bytes": (u64, [vp]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype, f.argtypes = res, args
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _bytes(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray)):
        return np.frombuffer(bytes(x), dtype=np.uint8).copy() if len(x) else np.zeros(1, np.uint8)
    a = np.ascontiguousarray(x, dtype=np.uint8)
    return a if a.size else np.zeros(1, np.uint8)


# ---- scalar helpers ---------------------------------------------------------

def mix64(x: int) -> int:
    return int(lib().orc_mix64(x))


def splitmix64(seed: int, n: int) -> list[int]:
    st = C.c_uint64(seed)
    return [int(lib().orc_splitmix64_next(C.byref(st))) for _ in range(n)]


def term_hash(term: int, seed: int, i: int) -> int:
    return int(lib().orc_term_hash(term, seed, i))


def terms(kind: int, q: int, canonical: bool, s) -> np.ndarray:
    b = _bytes(s)
    n = len(s)
    out = np.zeros(max(n, 1), np.uint64)
    k = lib().orc_terms(kind, q, int(canonical), _ptr(b), n, _ptr(out))
    return out[:k].copy()


def unique(a) -> np.ndarray:
    a = np.array(a, dtype=np.uint64, copy=True)
    k = lib().orc_unique(_ptr(a), a.size) if a.size else 0
    return a[:k].copy()


def filter_rows(n: int, h: int, p: float) -> int:
    return int(lib().orc_filter_rows(n, h, p))


def bloom_fpr(m: float, h: int, n: float) -> float:
    return float(lib().orc_bloom_fpr(m, h, n))


def bloom_fpr_exp(m: float, h: int, n: float) -> float:
    return float(lib().orc_bloom_fpr_exp(m, h, n))


def binom_tail_gt(l: int, p: float, f: int) -> float:
    return float(lib().orc_binom_tail_gt(l, p, f))


def chernoff(l: int, p: float, K: float) -> float:
    return float(lib().orc_chernoff(l, p, K))


# ---- documents --------------------------------------------------------------

class Docs:
    """Documents as CSR: doc d owns strings doc_str[d]..doc_str[d+1]; string s
    is bytes[str_off[s]:str_off[s+1]]."""

    def __init__(self, data: np.ndarray, str_off: np.ndarray, doc_str: np.ndarray):
        self.bytes = np.ascontiguousarray(data, dtype=np.uint8)
        self.str_off = np.ascontiguousarray(str_off, dtype=np.uint64)
        self.doc_str = np.ascontiguousarray(doc_str, dtype=np.uint64)
        self.n_docs = len(self.doc_str) - 1

    @classmethod
    def from_lists(cls, docs):
        """docs: list of documents, each a list of strings (bytes/str)."""
        chunks, str_off, doc_str = [], [0], [0]
        for d in docs:
            if isinstance(d, (bytes, str)):
                d = [d]
            for s in d:
                s = s.encode() if isinstance(s, str) else bytes(s)
                chunks.append(s)
                str_off.append(str_off[-1] + len(s))
            doc_str.append(len(str_off) - 1)
        data = np.frombuffer(b"".join(chunks), dtype=np.uint8).copy()
        return cls(data, np.array(str_off, np.uint64), np.array(doc_str, np.uint64))

    def _safe_bytes(self):
        return self.bytes if self.bytes.size else np.zeros(1, np.uint8)


class OracleIndex:
    """Classic (B=0) or compact (B>0) bit-sliced signature matrix."""

    def __init__(self, docs: Docs, kind=DNA, q=31, canonical=True, h=1, p=0.3,
                 B=0, seed=0, row_align=128):
        self.params = _Params(kind, q, int(canonical), h, p, B, seed, row_align)
        self.docs = docs
        self._data = docs._safe_bytes()
        self._h = lib().orc_build(C.byref(self.params), _ptr(self._data),
                                  _ptr(docs.str_off), _ptr(docs.doc_str), docs.n_docs)
        if not self._h:
            raise MemoryError("oracle index does not fit host memory")
        self.n_docs = docs.n_docs

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    @property
    def n_blocks(self) -> int:
        return int(lib().orc_n_blocks(self._h))

    def block(self, b: int) -> dict:
        f, d = C.c_uint32(), C.c_uint32()
        r, s, o = C.c_uint64(), C.c_uint64(), C.c_uint64()
        lib().orc_block_info(self._h, b, C.byref(f), C.byref(d), C.byref(r),
                             C.byref(s), C.byref(o))
        return dict(first=f.value, docs=d.value, rows=r.value, stride=s.value,
                    offset=o.value)

    def order(self) -> np.ndarray:
        p = lib().orc_order(self._h)
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint32)),
                                     (max(self.n_docs, 1),))[: self.n_docs].copy()

    def n_terms(self) -> np.ndarray:
        p = lib().orc_n_terms(self._h)
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint64)),
                                     (max(self.n_docs, 1),))[: self.n_docs].copy()

    def matrix(self) -> np.ndarray:
        n = int(lib().orc_total_bytes(self._h))
        if n == 0:
            return np.zeros(0, np.uint8)
        p = lib().orc_bits(self._h)
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint8)), (n,)).copy()

    def bit(self, b: int, row: int, j: int) -> int:
        return int(lib().orc_bit(self._h, b, row, j))

    def query_scores(self, query) -> tuple[np.ndarray, int]:
        qb = _bytes(query)
        scores = np.zeros(max(self.n_docs, 1), np.uint32)
        l = lib().orc_query_scores(self._h, _ptr(qb), len(query), _ptr(scores))
        return scores[: self.n_docs], int(l)

    def query(self, query, k_num=4, k_den=5, topk=0):
        scores, l = self.query_scores(query)
        return report(scores, l, k_num, k_den, topk) + (l,)

    def query_many(self, queries, threads: int = 1):
        """Score a list of queries, optionally on several threads (ctypes
        releases the GIL inside the C call)."""
        if threads <= 1:
            return [self.query_scores(q) for q in queries]
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            return list(ex.map(self.query_scores, queries))


def plan(n_terms, B: int):
    """Block plan of section 2.2/2.3 from per-document distinct-term counts:
    (order, [(first, docs, n_max) per block])."""
    n = np.ascontiguousarray(n_terms, dtype=np.uint64)
    nd = n.size
    order = np.zeros(max(nd, 1), np.uint32)
    nb_cap = max((nd + B - 1) // B if B else 1, 1)
    first = np.zeros(nb_cap, np.uint32)
    docs = np.zeros(nb_cap, np.uint32)
    nmax = np.zeros(nb_cap, np.uint64)
    nb = lib().orc_plan(_ptr(n if nd else np.zeros(1, np.uint64)), nd, B, _ptr(order),
                        _ptr(first), _ptr(docs), _ptr(nmax))
    return order[:nd].copy(), [(int(first[b]), int(docs[b]), int(nmax[b])) for b in range(nb)]


def report(scores: np.ndarray, l: int, k_num: int, k_den: int, topk: int):
    scores = np.ascontiguousarray(scores, dtype=np.uint32)
    n = scores.size
    ids = np.zeros(max(n, 1), np.uint32)
    sc = np.zeros(max(n, 1), np.uint32)
    k = lib().orc_report(_ptr(scores if n else np.zeros(1, np.uint32)), n, l,
                         k_num, k_den, topk, _ptr(ids), _ptr(sc))
    return ids[:k].copy(), sc[:k].copy()


def bruteforce_scores(docs: Docs, query, kind=DNA, q=31, canonical=True, h=1,
                      p=0.3, B=0, seed=0):
    prm = _Params(kind, q, int(canonical), h, p, B, seed, 128)
    qb = _bytes(query)
    out = np.zeros(max(docs.n_docs, 1), np.uint32)
    l = lib().orc_bruteforce_scores(C.byref(prm), _ptr(docs._safe_bytes()),
                                    _ptr(docs.str_off), _ptr(docs.doc_str),
                                    docs.n_docs, _ptr(qb), len(query), _ptr(out))
    return out[: docs.n_docs], int(l)


def exact_intersection(docs: Docs, query, kind=DNA, q=31, canonical=True):
    prm = _Params(kind, q, int(canonical), 1, 0.5, 0, 0, 128)
    qb = _bytes(query)
    out = np.zeros(max(docs.n_docs, 1), np.uint32)
    l = lib().orc_exact_intersection(C.byref(prm), _ptr(docs._safe_bytes()),
                                     _ptr(docs.str_off), _ptr(docs.doc_str),
                                     docs.n_docs, _ptr(qb), len(query), _ptr(out))
    return out[: docs.n_docs], int(l)


# ---- one document at a time --------------------------------------------------

class QuerySet:
    """Distinct terms of each query and their rows at a filter size m, for
    scoring documents one by one (block and column separability, section 2.2):
    a document's score depends only on its own terms, m and the query."""

    def __init__(self, queries, kind=DNA, q=31, canonical=True, h=1, p=0.3, seed=0):
        self.params = _Params(kind, q, int(canonical), h, p, 0, seed, 128)
        per = [unique(terms(kind, q, canonical, x)) for x in queries]
        self.ell = np.array([len(t) for t in per], np.uint64)
        self.off = np.zeros(len(per) + 1, np.uint64)
        np.cumsum(self.ell, out=self.off[1:])
        self.terms = np.concatenate(per).astype(np.uint64) if per else np.zeros(0, np.uint64)
        self.total = int(self.off[-1])
        self._rows = {}

    def rows(self, m: int) -> np.ndarray:
        if m not in self._rows:
            out = np.zeros(max(self.params.h * self.total, 1), np.uint64)
            src = self.terms if self.total else np.zeros(1, np.uint64)
            lib().orc_term_rows(C.byref(self.params), m, _ptr(src), self.total, _ptr(out))
            self._rows[m] = out
        return self._rows[m]

    def doc_scores(self, m: int, strings) -> np.ndarray:
        """Scores of the document made of `strings` at filter size m."""
        if isinstance(strings, np.ndarray):
            data = _bytes(strings)
            so = np.array([0, strings.size], np.uint64)
            n_str = 1
        else:
            if isinstance(strings, (bytes, bytearray)):
                strings = [strings]
            parts = [bytes(x) for x in strings]
            data = _bytes(b"".join(parts))
            so = np.zeros(len(parts) + 1, np.uint64)
            np.cumsum([len(x) for x in parts], out=so[1:])
            n_str = len(parts)
        nq = len(self.ell)
        out = np.zeros(max(nq, 1), np.uint32)
        rows = self.rows(m)
        lib().orc_doc_scores(C.byref(self.params), m, _ptr(data), _ptr(so), n_str, _ptr(rows),
                             self.total, _ptr(self.off), nq, _ptr(out))
        return out[:nq]


def rc_palindrome_dups(q: int, s) -> tuple[int, int]:
    """(windows of s repeating an earlier window as its reverse complement
    through a palindrome, valid windows) for canonical DNA q-mers."""
    b = _bytes(s)
    v = C.c_uint64()
    k = lib().orc_rc_palindrome_dups(q, _ptr(b), len(s), C.byref(v))
    return int(k), int(v.value)
