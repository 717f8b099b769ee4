"""Parity at the full sizes of the benchmark workloads.

The GPU builds the whole index (DNA: documents generated in device memory
and the streamed two-pass build the benchmark uses; text: the one-call build
from host bytes) and scores queries against every document in the
benchmark's launch shapes.  The oracle cannot build a 54 GB index, but a
document's score depends only on its own terms, its block's row count m_b
and the query (block and column separability, section 2.2), so it scores
documents one at a time (oracle.QuerySet.doc_scores) and checks:

* the plan: every document's distinct-term count from a source independent
  of the GPU.  Text: the oracle counts every document.  DNA: a uniform-random
  ACGT document of length L has L - 30 windows; its canonical 31-mers repeat
  almost only where a window is the reverse complement of an overlapping one
  (a hairpin of 32 or more bases, about once in 4^16 positions), which the
  oracle's palindrome scan finds exactly in every document; any document
  whose GPU count differs from L - 30 minus those repeats is recounted
  exactly by the oracle (sort and unique of its terms).  The expected order,
  blocks and row counts follow from those counts.
* whole blocks, column by column: every document of the checked blocks
  (compact-100k: the first block of 8,192 and the last, narrow block of
  1,696; text-50k: one block of 8,192 at h = 3; classic-10k: 1,024
  contiguous columns and the 1,808 of its 256-byte second slice) plus two
  sampled documents and the largest of every other block.  Full score
  vectors, the K = 4/5 hits restricted to those documents, and the top-100
  lists (consistent with the full scores, which are checked on those
  documents) must match.  With early exit of threshold queries (cobs_prune)
  the K = 4/5 and K = 1 hits must equal the unpruned hits for every document.
* serving at full size (the compact 100k index): requests of the serving
  mix (31 bp to 1 Mbp), replayed as Poisson arrivals through a 4-stream
  server, get the batch path's hits, whose scores match the oracle on the
  checked documents.
"""
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

THREADS = 16


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    return torch, cobs


def _log(msg):
    print(f"[fullsize {time.strftime('%H:%M:%S')}] {msg}", flush=True)


class _Docs:
    """Bytes of single documents of a workload, by input id."""

    def __init__(self, w, host=None):
        self.w, self.host = w, host
        self.lens = synth.doc_lengths(w)

    def get(self, d):
        """The document's bytes (a uint8 array)."""
        if self.host is not None:
            return self.host.bytes[int(self.host.str_off[d]):int(self.host.str_off[d + 1])]
        n = int(self.lens[d])
        out = np.empty(max(n, 1), np.uint8)
        if n:
            synth.lib().synth_doc_bases(self.w.seed, d, 0, n, synth._p(out))
        return out[:n]


def _kind(w):
    return oracle.DNA if w.kind == "dna" else oracle.BYTES


def _exact_count(w, text):
    return len(oracle.unique(oracle.terms(_kind(w), w.q, w.canonical, text)))


def _expected_counts(w, docs, gpu_counts):
    """Distinct-term counts of every document, independent of the GPU's."""
    ids = range(w.n_docs)
    if w.kind != "dna":
        with ThreadPoolExecutor(THREADS) as ex:
            return np.array(list(ex.map(lambda d: _exact_count(w, docs.get(d)), ids)), np.int64), w.n_docs

    def scan(d):
        dups, valid = oracle.rc_palindrome_dups(w.q, docs.get(d))
        return valid - dups

    with ThreadPoolExecutor(THREADS) as ex:
        n_exp = np.array(list(ex.map(scan, ids, chunksize=64)), np.int64)
    hairpins = int((n_exp < np.maximum(docs.lens.astype(np.int64) - (w.q - 1), 0)).sum())
    recount = np.nonzero(gpu_counts.astype(np.int64) != n_exp)[0]
    _log(f"{w.name}: {hairpins} documents with reverse-complement repeats; "
         f"{len(recount)} recounted exactly")
    assert len(recount) <= 8, len(recount)
    for d in recount:
        n_exp[d] = _exact_count(w, docs.get(int(d)))
    return n_exp, len(recount)


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
    assert np.array_equal(n_terms.astype(np.int64), n_exp)
    ids = np.arange(w.n_docs)
    order_exp = np.lexsort((ids, n_exp)) if w.B else ids
    assert np.array_equal(order.astype(np.int64), order_exp)
    return order, n_exp


def _columns(w, ix, order, n_exp, whole, per_block, rng):
    """(rows, member ids) per block: every document of the blocks in `whole`
    (a block index, or (block, [sorted positions]) for part of one), else
    per_block sampled documents plus the block's largest."""
    whole = dict((x, None) if isinstance(x, int) else x for x in whole)
    groups = []
    for b in range(ix.info()["n_blocks"]):
        blk = ix.block(b)
        first, n = blk["first"], blk["docs"]
        assert n == (min(w.B, w.n_docs - first) if w.B else w.n_docs)
        members = order[first:first + n].astype(np.int64)
        big = int(np.argmax(n_exp[members]))    # the last one when size-sorted
        assert blk["rows"] == oracle.filter_rows(int(n_exp[members[big]]), w.h, w.p)
        if b in whole:
            pos = np.arange(n) if whole[b] is None else np.asarray(whole[b])
        else:
            others = np.delete(np.arange(n), big)
            pos = np.append(rng.choice(others, size=min(per_block, len(others)), replace=False), big)
        groups.append((blk["rows"], [int(members[p]) for p in pos]))
    return groups


def _oracle_columns(w, docs, groups, qset):
    """Oracle scores [n_queries, n_docs] on the checked documents (others -1)."""
    out = np.full((len(qset.ell), w.n_docs), -1, np.int64)
    jobs = [(rows, d) for rows, ids in groups for d in ids]
    done = [0]
    t0 = time.time()

    def one(job):
        rows, d = job
        out[:, d] = qset.doc_scores(rows, docs.get(d))
        done[0] += 1
        if done[0] % 2000 == 0:
            _log(f"oracle: {done[0]}/{len(jobs)} documents ({time.time() - t0:.0f}s)")

    with ThreadPoolExecutor(THREADS) as ex:
        list(ex.map(one, jobs, chunksize=8))
    _log(f"oracle: {len(jobs)} documents scored in {time.time() - t0:.0f}s")
    return out


def _checked(groups):
    return np.array(sorted(d for _, ids in groups for d in ids), np.int64)


def _compare_scores(want, sc, nt, ell, cols, label):
    assert np.array_equal(nt.astype(np.int64), ell.astype(np.int64)), label
    bad = np.nonzero((sc[:, cols].astype(np.int64) != want[:, cols]).any(axis=1))[0]
    assert len(bad) == 0, (label, bad[:5])


def _compare_hits(want, hits, ell, cols, k):
    """K = k[0]/k[1] hits restricted to the checked documents."""
    colset = np.zeros(want.shape[1], bool)
    colset[cols] = True
    for qi, (ids, scores, l) in enumerate(hits):
        assert l == ell[qi]
        T = -(-k[0] * int(ell[qi]) // k[1])
        keep = colset[ids.astype(np.int64)]
        got = sorted(zip((-scores[keep].astype(np.int64)).tolist(), ids[keep].astype(np.int64).tolist()))
        if ell[qi] == 0:
            exp = []
        else:
            sel = cols[want[qi, cols] >= T]
            exp = sorted(zip((-want[qi, sel]).tolist(), sel.tolist()))
        assert got == exp, qi


def _check_topk(sc, hits, topk):
    """top-k lists = the first top-k of (score desc, id asc) of the full scores."""
    for qi, (ids, scores, l) in enumerate(hits):
        row = sc[qi].astype(np.int64)
        if l == 0:
            assert len(ids) == 0
            continue
        exp = np.lexsort((np.arange(row.size), -row))[:topk]
        assert np.array_equal(ids.astype(np.int64), exp), qi
        assert np.array_equal(scores.astype(np.int64), row[exp]), qi


def _check_full_size(w, ix, docs, whole, per_block, queries, shapes, rng, topk=0):
    order, n_exp = _check_plan(w, ix, docs)
    _log(f"{w.name}: plan checked")
    groups = _columns(w, ix, order, n_exp, whole, per_block, rng)
    cols = _checked(groups)
    data, off = _pack(queries)
    gpu = []
    for unroll, cap in shapes:
        ix.set_tuning(unroll, cap)
        gpu.append(ix.scores(data, off))
    ix.set_tuning(0, 0)
    hits = ix.query(data, off, k=w.k)
    top = ix.query(data, off, k=(0, 1), topk=topk) if topk else None
    # early exit of threshold queries: the same hits for every document, at
    # the workload's K and at K = 1 (T = l: only documents holding every
    # term counted so far stay live)
    full1 = ix.query(data, off, k=(1, 1))
    ix.set_tuning(prune=1)
    phits = ix.query(data, off, k=w.k)
    pfull1 = ix.query(data, off, k=(1, 1))
    ix.set_tuning(0, 0)
    for qi, (a, b) in enumerate(list(zip(hits, phits)) + list(zip(full1, pfull1))):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2], qi
    _log(f"{w.name}: GPU scores of {len(queries)} queries in {len(shapes)} launch shapes")
    qset = oracle.QuerySet(queries, kind=_kind(w), q=w.q, canonical=w.canonical, h=w.h, p=w.p,
                           seed=w.hash_seed)
    want = _oracle_columns(w, docs, groups, qset)
    for (sc, nt), shape in zip(gpu, shapes):
        _compare_scores(want, sc, nt, qset.ell, cols, shape)
    _compare_hits(want, hits, qset.ell, cols, w.k)
    _compare_hits(want, phits, qset.ell, cols, w.k)
    if top is not None:
        _check_topk(gpu[0][0], top, topk)
    return groups, n_exp, gpu[0], want, qset


def test_compact_100k_full_size_whole_blocks_and_served():
    # 100,000 documents, 13 blocks of up to 8,192, 54 GB; the benchmark's
    # launch shapes: unroll 4 or 8, chunk cap 16384 or one item per query
    torch, cobs = _gpu()
    import bench
    w = synth.CONFIGS[3]
    ix = bench.build_index_dna(cobs, synth, torch, w, 8 << 30)
    docs = _Docs(w)
    rng = np.random.default_rng(3)
    qs = synth.dna_queries(w, n=120)
    bench_q = [qs.get(i) for i in range(qs.n)]
    # planted queries from documents of the first and the last block
    lens = docs.lens.astype(np.int64)
    by_size = np.argsort(lens, kind="stable")
    sources = [int(x) for x in list(by_size[:4]) + list(by_size[-4:])]
    planted = _planted(rng, [docs.get(d).tobytes() for d in sources], 16, 2000)
    # the serving mix: 40 requests of 31 bp .. 1 Mbp
    w5 = synth.CONFIGS[5]
    pool = synth.dna_queries(w5, n=40)
    pool_q = [pool.get(i) for i in range(pool.n)]
    queries = bench_q + planted + pool_q
    n_last = ix.info()["n_blocks"] - 1
    groups, n_exp, (sc, nt), want, qset = _check_full_size(
        w, ix, docs, [0, n_last], 2, queries, [(4, 16384), (8, 1 << 20)], rng, topk=100)
    assert len(groups[0][1]) == 8192 and len(groups[n_last][1]) == 1696
    # the planted queries find their source document at a full score
    for j, d in enumerate(sources * 2):
        qi = len(bench_q) + j
        assert sc[qi, d] == nt[qi]

    # serving at full size, as the benchmark serves: every result equals the
    # batch path's, whose scores were checked above
    data, off = _pack(pool_q)
    batch = ix.query(data, off, k=w5.k)
    srv = cobs.Server(ix, num_streams=4)
    lat, nh = srv.replay(data, off, synth.arrivals(5, pool.n, 200.0), k=w5.k)
    st = srv.stop()
    assert st["completed"] == pool.n and np.all(lat > 0)
    assert list(nh) == [len(b[0]) for b in batch]
    srv = cobs.Server(ix, num_streams=4)
    tickets = [srv.submit(q, k=w5.k) for q in pool_q]
    served = [srv.wait(t) for t in tickets]
    srv.stop()
    for s, b in zip(served, batch):
        assert np.array_equal(s[0], b[0]) and np.array_equal(s[1], b[1]) and s[2] == b[2]
    base = len(bench_q) + len(planted)
    _compare_hits(want[base:], batch, qset.ell[base:], _checked(groups), w5.k)

    # out of core at full size: the matrix in pinned host memory, the bench
    # and planted queries read in place (their rows are far fewer than the
    # matrix), scores and hits against the oracle on the checked documents
    data, off = _pack(bench_q + planted)
    n_q = len(bench_q) + len(planted)
    ix.offload(30 * 10**9)
    assert ix.info()["host_resident"]
    ix.set_tuning(host_reads=cobs.HOST_READS_IN_PLACE)
    osc, ont = ix.scores(data, off)
    _compare_scores(want[:n_q], osc, ont, qset.ell[:n_q], _checked(groups), "in place")
    _compare_hits(want[:n_q], ix.query(data, off, k=w.k), qset.ell[:n_q], _checked(groups), w.k)
    ix.set_tuning()


def test_classic_10k_full_size_columns():
    # 10,000 documents in one block of 2.8 M rows x 1,280 bytes: the first
    # 1,024 columns and the whole second slice (256 bytes, documents 8,192 ..
    # 9,999)
    torch, cobs = _gpu()
    import bench
    w = synth.CONFIGS[2]
    ix = bench.build_index_dna(cobs, synth, torch, w, 8 << 30)
    qs = synth.dna_queries(w, n=120)
    docs = _Docs(w)
    rng = np.random.default_rng(2)
    planted = _planted(rng, [docs.get(d).tobytes() for d in (3, 700, 8200, 9999)], 8, 2000)
    part = list(range(1024)) + list(range(8192, w.n_docs))
    groups, *_ = _check_full_size(w, ix, docs, [(0, part)], 0,
                                  [qs.get(i) for i in range(qs.n)] + planted, [(8, 16384)], rng)
    assert groups[0][1] == part


def test_text_50k_full_size_whole_block():
    # 50,000 text documents, 7 blocks, h = 3 (every document counted by the
    # oracle); block 5 (8,192 documents) whole, gathered by the unpacked
    # h = 3 instantiation
    torch, cobs = _gpu()
    w = synth.CONFIGS[4]
    d = synth.docs(w)
    prm = cobs.make_params(cobs.BYTES, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    assert ix.block(5)["docs"] == 8192 and ix.block(5)["stride"] == 1024
    qs = synth.text_queries(w, d, n=150)
    _check_full_size(w, ix, _Docs(w, d), [5], 2, [qs.get(i) for i in range(qs.n)],
                     [(4, 8192), (2, 1 << 20)], np.random.default_rng(4))
