"""Querying several indexes as one collection (cobs_query_multi): each
document's score is the one the oracle gives it in its own index, documents
are numbered across the indexes in order, hits over all of them come in
(score desc, global id asc) order and top-k keeps the best over the union;
for indexes that can be merged the result is the merged index's."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _cobs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    return cobs


def rand_dna(rng, n):
    return rng.choice(np.frombuffer(b"ACGT", np.uint8), n).tobytes()


def _build(cobs, docs, h, p, B, seed):
    d = oracle.Docs.from_lists(docs)
    prm = cobs.make_params(0, 31, True, h, p, B, seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    oix = oracle.OracleIndex(d, kind=0, q=31, canonical=True, h=h, p=p, B=B, seed=seed)
    return ix, oix


def _queries(rng, parts):
    qs = []
    for docs in parts:
        qs += [docs[i][50:50 + int(rng.integers(31, 1500))] for i in range(0, len(docs), 4)]
    qs += [rand_dna(rng, 900) for _ in range(4)] + [b"", b"ACGT" * 5]
    off = np.zeros(len(qs) + 1, np.uint64)
    np.cumsum([len(q) for q in qs], out=off[1:])
    return qs, np.frombuffer(b"".join(qs), np.uint8), off


def _want(oixs, q, k_num, k_den, topk):
    """The oracle: scores in each index, concatenated in index order, then
    the threshold and the (score desc, global id asc) order."""
    parts = [o.query_scores(q) for o in oixs]
    ells = {l for _, l in parts}
    assert len(ells) == 1
    ell = ells.pop()
    sc = np.concatenate([s for s, _ in parts]).astype(np.int64)
    if ell == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), 0
    T = -(-k_num * ell // k_den)
    ids = np.nonzero(sc >= T)[0]
    ids = ids[np.lexsort((ids, -sc[ids]))]
    if topk:
        ids = ids[:topk]
    return ids, sc[ids], ell


@pytest.fixture(scope="module")
def parts():
    cobs = _cobs()
    rng = np.random.default_rng(31)
    A = [rand_dna(rng, int(rng.integers(800, 6000))) for _ in range(23)]
    B = [rand_dna(rng, int(rng.integers(800, 9000))) for _ in range(37)]
    C = [rand_dna(rng, int(rng.integers(800, 4000))) for _ in range(11)]
    # different h, p, seed and block size; one term definition
    built = [_build(cobs, A, 1, 0.3, 8, 7), _build(cobs, B, 2, 0.2, 16, 99),
             _build(cobs, C, 3, 0.1, 0, 5)]
    return cobs, rng, (A, B, C), built


@pytest.mark.parametrize("k,topk,mode", [((1, 2), 0, 0), ((0, 1), 0, 0), ((0, 1), 7, 0),
                                         ((3, 4), 2, 0), ((1, 2), 5, 1)])
def test_multi_equals_oracle_over_the_union(parts, k, topk, mode):
    cobs, rng, docs, built = parts
    qs, data, off = _queries(rng, docs)
    ixs = [ix for ix, _ in built]
    oixs = [o for _, o in built]
    got = cobs.query_multi(ixs, data, off, k=k, topk=topk, mode=mode)
    assert len(got) == len(qs)
    for i, q in enumerate(qs):
        ids, sc, l = _want(oixs, q, k[0], k[1], topk)
        assert got[i][2] == l, i
        assert np.array_equal(got[i][0], ids) and np.array_equal(got[i][1], sc), (i, k, topk)


def test_multi_with_early_exit_equals_oracle(parts):
    # every index with early exit on: the same union of hits
    cobs, rng, docs, built = parts
    qs, data, off = _queries(rng, docs)
    ixs = [ix for ix, _ in built]
    oixs = [o for _, o in built]
    for ix in ixs:
        ix.set_tuning(prune=cobs.PRUNE_ON)
    try:
        for k, topk, chunk in (((3, 4), 2, 0), ((4, 5), 0, 32)):
            got = cobs.query_multi(ixs, data, off, k=k, topk=topk, chunk=chunk)
            for i, q in enumerate(qs):
                ids, sc, l = _want(oixs, q, k[0], k[1], topk)
                assert got[i][2] == l, i
                assert np.array_equal(got[i][0], ids) and np.array_equal(got[i][1], sc), (i, k, topk)
    finally:
        for ix in ixs:
            ix.set_tuning()


def test_multi_of_one_index_is_the_index(parts):
    cobs, rng, docs, built = parts
    qs, data, off = _queries(rng, docs)
    ix = built[1][0]
    assert cobs.query_multi([ix, built[0][0]], b"", np.zeros(1, np.uint64)) == []   # no queries
    for k, topk in (((1, 2), 0), ((0, 1), 3)):
        for x, y in zip(cobs.query_multi([ix], data, off, k=k, topk=topk),
                        ix.query(data, off, k=k, topk=topk)):
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) and x[2] == y[2]


def test_multi_equals_the_merged_index():
    import torch
    cobs = _cobs()
    rng = np.random.default_rng(32)
    A = [rand_dna(rng, int(rng.integers(1000, 7000))) for _ in range(19)]
    B = [rand_dna(rng, int(rng.integers(1000, 7000))) for _ in range(26)]
    ia, _ = _build(cobs, A, 1, 0.3, 8, 7)
    ib, _ = _build(cobs, B, 1, 0.3, 8, 7)
    merged = ia.merge(ib)
    qs, data, off = _queries(rng, [A, B])
    ddata = torch.from_numpy(data.copy()).to("cuda")          # query bytes in device memory
    for k, topk in (((1, 2), 0), ((0, 1), 10), ((4, 5), 1)):
        for x, y in zip(cobs.query_multi([ia, ib], ddata, off, k=k, topk=topk),
                        merged.query(data, off, k=k, topk=topk)):
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) and x[2] == y[2]
    # one part kept in host memory and streamed, the other in HBM
    big = max(ib.block(b)["rows"] * ib.block(b)["stride"] for b in range(ib.info()["n_blocks"]))
    ib.offload(2 * ((big + 255) // 256 * 256))
    try:
        for x, y in zip(cobs.query_multi([ia, ib], data, off, k=(1, 2)), merged.query(data, off, k=(1, 2))):
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) and x[2] == y[2]
    finally:
        ib.onload()


def test_multi_refuses_mixed_term_definitions(parts):
    cobs, rng, docs, built = parts
    qs, data, off = _queries(rng, docs)
    d = oracle.Docs.from_lists(docs[0])
    other = cobs.Index.build(cobs.make_params(0, 25, True, 1, 0.3, 8, 7), d.bytes, d.str_off,
                             d.doc_str)
    for bad in ([built[0][0], other], []):
        with pytest.raises(cobs.CobsError) as e:
            cobs.query_multi(bad, data, off)
        assert e.value.status == cobs.EINVAL
