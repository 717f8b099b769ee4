"""Parity at the full sizes of the benchmark workloads, on sampled outputs.

The GPU builds the whole index (documents generated in device memory, the
streamed two-pass build the benchmark uses) and scores queries against every
document in the benchmark's launch shapes.  The oracle cannot build a 54 GB
index, so it checks what it can compute one by one:

* the plan: a uniform-random ACGT document of length L has L - 30 distinct
  canonical 31-mers unless two of its windows share a canonical form.  Far
  apart that is rare (about L^2 / 4^31), but a window and the next one are
  reverse complements of each other when 16 base pairs match (a hairpin,
  about one position in 4^16), so a few dozen of the 1.3 * 10^11 windows of
  the compact 100k set do it.  The oracle counts every document whose GPU
  count differs from L - 30 exactly (there must be only a few), and the
  sampled documents; the expected order and blocks follow from those counts.
* the scores of sampled documents: per block, an oracle index over the
  sampled documents plus the block's largest one (classic layout, so its
  row count is the block's m_b) gives each sampled document's score for
  every query; the GPU's full score matrix must match it exactly.
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


def _exact_count(w, d):
    text = synth.dna_docs(w, first=d, count=1).bytes.tobytes()
    return len(oracle.unique(oracle.terms(oracle.DNA, w.q, w.canonical, text)))


def _expected_plan(w, gpu_counts):
    lens = synth.doc_lengths(w).astype(np.int64)
    n_terms = np.maximum(lens - (w.q - 1), 0)
    recount = np.nonzero(gpu_counts.astype(np.int64) != n_terms)[0]
    assert len(recount) <= 64, len(recount)
    for d in recount:
        n_terms[d] = _exact_count(w, int(d))
    ids = np.arange(len(n_terms))
    order = np.lexsort((ids, n_terms)) if w.B else ids
    return n_terms, order, len(recount)


def _planted(rng, docs, n, length):
    out = []
    for i in range(n):
        d = docs[i % len(docs)]
        a = int(rng.integers(0, max(1, len(d) - length)))
        out.append(d[a:a + length])
    return out


def _check_full_size(w, samples_per_block, n_bench_queries, shapes):
    torch, cobs = _gpu()
    import bench
    ix = bench.build_index_dna(cobs, synth, torch, w, 8 << 30)
    order, n_terms = ix.order()
    n_exp, order_exp, recounted = _expected_plan(w, n_terms)
    print(f"{recounted} documents recounted by the oracle")
    assert np.array_equal(n_terms.astype(np.int64), n_exp)
    assert np.array_equal(order.astype(np.int64), order_exp)
    info = ix.info()
    rng = np.random.default_rng(w.seed & 0xFFFF)
    groups = []   # (block rows, sampled ids, id of the block's largest document)
    for b in range(info["n_blocks"]):
        blk = ix.block(b)
        first, docs = blk["first"], blk["docs"]
        assert docs == (min(w.B, w.n_docs - first) if w.B else w.n_docs)
        members = order[first:first + docs].astype(np.int64)
        big = int(np.argmax(n_exp[members]))    # the last one when size-sorted
        assert blk["rows"] == oracle.filter_rows(int(n_exp[members[big]]), w.h, w.p)
        others = np.delete(np.arange(docs), big)
        pos = rng.choice(others, size=min(samples_per_block, len(others)), replace=False)
        groups.append((blk["rows"], [int(members[p]) for p in pos], int(members[big])))

    # queries: the benchmark's first queries, plus exact substrings of sampled documents
    qs = synth.dna_queries(w, n=n_bench_queries)
    queries = [qs.get(i) for i in range(qs.n)]
    some = [g[1][0] for g in groups[:8]]
    some_bytes = [synth.dna_docs(w, first=d, count=1).bytes.tobytes() for d in some]
    queries += _planted(rng, some_bytes, 16, 2000)
    off = np.zeros(len(queries) + 1, np.uint64)
    np.cumsum([len(q) for q in queries], out=off[1:])
    data = np.frombuffer(b"".join(queries), np.uint8)

    gpu = []
    for unroll, cap in shapes:
        ix.set_tuning(unroll, cap)
        gpu.append(ix.scores(data, off))
    ix.set_tuning(0, 0)

    def oracle_block(g):
        rows, ids, last = g
        members = ids + [last]
        texts = [synth.dna_docs(w, first=d, count=1).bytes.tobytes() for d in members]
        oix = oracle.OracleIndex(oracle.Docs.from_lists(texts), kind=oracle.DNA, q=w.q,
                                 canonical=w.canonical, h=w.h, p=w.p, B=0,
                                 seed=w.hash_seed, row_align=1)
        assert np.array_equal(oix.n_terms().astype(np.int64), n_exp[members])
        assert oix.block(0)["rows"] == rows
        res = [oix.query_scores(q) for q in queries]
        del oix
        return members, res

    with ThreadPoolExecutor(8) as ex:
        for members, res in ex.map(oracle_block, groups):
            for qi, (want, wl) in enumerate(res):
                for sc, nt in gpu:
                    assert nt[qi] == wl, qi
                    # every sampled document, and the block's largest one
                    assert np.array_equal(sc[qi, members], want), (qi, members)
    # the planted queries find their source document at a full score
    for j, d in enumerate(some * 2):
        qi = n_bench_queries + j
        for sc, nt in gpu:
            assert sc[qi, d] == nt[qi]


def test_compact_100k_full_size_sampled():
    # 100,000 documents, 13 blocks of up to 8,192, 54 GB; the benchmark's
    # launch shapes: unroll 4 or 8, chunk cap 16384 or one item per query
    _check_full_size(synth.CONFIGS[3], 2, 120, [(4, 16384), (8, 1 << 20)])


def test_classic_10k_full_size_sampled():
    # 10,000 documents in one block of 2.8 M rows x 1,280 bytes
    _check_full_size(synth.CONFIGS[2], 12, 120, [(8, 16384)])
