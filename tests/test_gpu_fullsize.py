"""Parity at the full sizes of the benchmark workloads, on sampled outputs.

The GPU builds the whole index (DNA: documents generated in device memory
and the streamed two-pass build the benchmark uses; text: the one-call build
from host bytes) and scores queries against every document in the
benchmark's launch shapes.  The oracle cannot build a 54 GB index, so it
checks what it can compute one by one:

* the plan.  Text: the oracle counts every document's distinct 8-grams.
  DNA: a uniform-random ACGT document of length L has L - 30 distinct
  canonical 31-mers unless two of its windows share a canonical form.  Far
  apart that is rare (about L^2 / 4^31), but a window and the next one are
  reverse complements of each other when 16 base pairs match (a hairpin,
  about one position in 4^16), so a few dozen of the 1.3 * 10^11 windows of
  the compact 100k set do it.  The oracle counts every document whose GPU
  count differs from L - 30 exactly (there must be only a few).  The
  expected order, blocks and row counts follow from those counts.
* the scores of sampled documents: per block, an oracle index over the
  sampled documents plus the block's largest one (classic layout, so its
  row count is the block's m_b) gives each sampled document's score for
  every query; the GPU's full score matrix must match it exactly.
* serving at full size (the compact 100k index): requests of the serving
  mix (31 bp to 1 Mbp), replayed as Poisson arrivals through a 4-stream
  server, get the batch path's hits, whose scores match the oracle on the
  sampled documents.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    return torch, cobs


class _Docs:
    """Bytes of single documents of a workload, by input id."""

    def __init__(self, w, host=None):
        self.w, self.host = w, host

    def get(self, d):
        if self.host is not None:
            return self.host.bytes[int(self.host.str_off[d]):int(self.host.str_off[d + 1])].tobytes()
        return synth.dna_docs(self.w, first=d, count=1).bytes.tobytes()


def _count(w, text):
    kind = oracle.DNA if w.kind == "dna" else oracle.BYTES
    return len(oracle.unique(oracle.terms(kind, w.q, w.canonical, text)))


def _expected_counts(w, docs, gpu_counts):
    if w.kind != "dna":
        with ThreadPoolExecutor(16) as ex:
            return np.array(list(ex.map(lambda d: _count(w, docs.get(d)), range(w.n_docs))),
                            np.int64), w.n_docs
    lens = synth.doc_lengths(w).astype(np.int64)
    n_terms = np.maximum(lens - (w.q - 1), 0)
    recount = np.nonzero(gpu_counts.astype(np.int64) != n_terms)[0]
    assert len(recount) <= 64, len(recount)
    for d in recount:
        n_terms[d] = _count(w, docs.get(int(d)))
    return n_terms, len(recount)


def _planted(rng, texts, n, length):
    out = []
    for i in range(n):
        t = texts[i % len(texts)]
        a = int(rng.integers(0, max(1, len(t) - length)))
        out.append(t[a:a + length])
    return out


def _pack(queries):
    off = np.zeros(len(queries) + 1, np.uint64)
    np.cumsum([len(q) for q in queries], out=off[1:])
    return np.frombuffer(b"".join(queries), np.uint8), off


def _check_plan(w, ix, docs):
    order, n_terms = ix.order()
    n_exp, counted = _expected_counts(w, docs, n_terms)
    print(f"{w.name}: {counted} documents counted by the oracle")
    assert np.array_equal(n_terms.astype(np.int64), n_exp)
    ids = np.arange(w.n_docs)
    order_exp = np.lexsort((ids, n_exp)) if w.B else ids
    assert np.array_equal(order.astype(np.int64), order_exp)
    return order, n_exp


def _sample_blocks(w, ix, order, n_exp, per_block, rng):
    groups = []   # (block rows, sampled ids, id of the block's largest document)
    for b in range(ix.info()["n_blocks"]):
        blk = ix.block(b)
        first, n = blk["first"], blk["docs"]
        assert n == (min(w.B, w.n_docs - first) if w.B else w.n_docs)
        members = order[first:first + n].astype(np.int64)
        big = int(np.argmax(n_exp[members]))    # the last one when size-sorted
        assert blk["rows"] == oracle.filter_rows(int(n_exp[members[big]]), w.h, w.p)
        others = np.delete(np.arange(n), big)
        pos = rng.choice(others, size=min(per_block, len(others)), replace=False)
        groups.append((blk["rows"], [int(members[p]) for p in pos], int(members[big])))
    return groups


def _oracle_scores(w, docs, groups, n_exp, queries):
    """Per block: (member ids, [(scores over members, l) per query])."""
    kind = oracle.DNA if w.kind == "dna" else oracle.BYTES

    def one(g):
        rows, ids, big = g
        members = ids + [big]
        oix = oracle.OracleIndex(oracle.Docs.from_lists([docs.get(d) for d in members]),
                                 kind=kind, q=w.q, canonical=w.canonical, h=w.h, p=w.p, B=0,
                                 seed=w.hash_seed, row_align=1)
        assert np.array_equal(oix.n_terms().astype(np.int64), n_exp[members])
        assert oix.block(0)["rows"] == rows
        res = [oix.query_scores(q) for q in queries]
        del oix
        return members, res

    with ThreadPoolExecutor(8) as ex:
        return list(ex.map(one, groups))


def _compare(oracle_res, gpu):
    for members, res in oracle_res:
        for qi, (want, wl) in enumerate(res):
            for sc, nt in gpu:
                assert nt[qi] == wl, qi
                # every sampled document, and the block's largest one
                assert np.array_equal(sc[qi, members], want), (qi, members)


def _check_full_size(w, ix, docs, per_block, bench_queries, shapes, rng):
    order, n_exp = _check_plan(w, ix, docs)
    groups = _sample_blocks(w, ix, order, n_exp, per_block, rng)
    some = [g[1][0] for g in groups[:8]]
    texts = [docs.get(d) for d in some]
    planted = _planted(rng, texts, 16, 2000 if w.kind == "dna" else 500)
    queries = bench_queries + planted
    data, off = _pack(queries)
    gpu = []
    for unroll, cap in shapes:
        ix.set_tuning(unroll, cap)
        gpu.append(ix.scores(data, off))
    ix.set_tuning(0, 0)
    _compare(_oracle_scores(w, docs, groups, n_exp, queries), gpu)
    # the planted queries find their source document at a full score
    for j, d in enumerate(some * 2):
        qi = len(bench_queries) + j
        for sc, nt in gpu:
            assert sc[qi, d] == nt[qi]
    return groups, n_exp


def test_compact_100k_full_size_sampled_and_served():
    # 100,000 documents, 13 blocks of up to 8,192, 54 GB; the benchmark's
    # launch shapes: unroll 4 or 8, chunk cap 16384 or one item per query
    torch, cobs = _gpu()
    import bench
    w = synth.CONFIGS[3]
    ix = bench.build_index_dna(cobs, synth, torch, w, 8 << 30)
    docs = _Docs(w)
    rng = np.random.default_rng(3)
    qs = synth.dna_queries(w, n=120)
    groups, n_exp = _check_full_size(w, ix, docs, 2, [qs.get(i) for i in range(qs.n)],
                                     [(4, 16384), (8, 1 << 20)], rng)

    # serving mix at full size: 40 requests of 31 bp .. 1 Mbp through a
    # 4-stream server, as the benchmark serves them
    w5 = synth.CONFIGS[5]
    pool = synth.dna_queries(w5, n=40)
    batch = ix.query(pool.bytes, pool.q_off, k=w5.k)
    srv = cobs.Server(ix, num_streams=4)
    lat, nh = srv.replay(pool.bytes, pool.q_off, synth.arrivals(5, pool.n, 200.0), k=w5.k)
    st = srv.stop()
    assert st["completed"] == pool.n and np.all(lat > 0)
    assert list(nh) == [len(b[0]) for b in batch]
    srv = cobs.Server(ix, num_streams=4)
    tickets = [srv.submit(pool.get(i), k=w5.k) for i in range(pool.n)]
    served = [srv.wait(t) for t in tickets]
    srv.stop()
    for s, b in zip(served, batch):
        assert np.array_equal(s[0], b[0]) and np.array_equal(s[1], b[1]) and s[2] == b[2]
    sc = ix.scores(pool.bytes, pool.q_off)
    queries = [pool.get(i) for i in range(pool.n)]
    _compare(_oracle_scores(w, docs, groups, n_exp, queries), [sc])


def test_classic_10k_full_size_sampled():
    # 10,000 documents in one block of 2.8 M rows x 1,280 bytes
    torch, cobs = _gpu()
    import bench
    w = synth.CONFIGS[2]
    ix = bench.build_index_dna(cobs, synth, torch, w, 8 << 30)
    qs = synth.dna_queries(w, n=120)
    _check_full_size(w, ix, _Docs(w), 12, [qs.get(i) for i in range(qs.n)], [(8, 16384)],
                     np.random.default_rng(2))


def test_text_50k_full_size_sampled():
    # 50,000 text documents, 7 blocks, h = 3 (every document counted by the oracle)
    torch, cobs = _gpu()
    w = synth.CONFIGS[4]
    d = synth.docs(w)
    prm = cobs.make_params(cobs.BYTES, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    qs = synth.text_queries(w, d, n=150)
    _check_full_size(w, ix, _Docs(w, d), 2, [qs.get(i) for i in range(qs.n)],
                     [(4, 8192), (2, 1 << 20)], np.random.default_rng(4))
