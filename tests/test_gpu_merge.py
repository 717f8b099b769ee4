"""Merging indexes (cobs_index_merge): classic indexes with equal row counts
concatenate row by row into exactly the index of the union; compact indexes
concatenate their blocks, and every document keeps the score it has in its
own index (checked against the oracle on each part)."""
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


def _build(cobs, docs, B):
    d = oracle.Docs.from_lists(docs)
    prm = cobs.make_params(0, 31, True, 1, 0.3, B, 7)
    return cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str), d


def _queries(rng, docs):
    qs = [docs[i][100:1100] for i in range(0, len(docs), 5)] + [rand_dna(rng, 800) for _ in range(5)]
    off = np.zeros(len(qs) + 1, np.uint64)
    np.cumsum([len(q) for q in qs], out=off[1:])
    return qs, np.frombuffer(b"".join(qs), np.uint8), off


def test_classic_merge_is_the_index_of_the_union():
    cobs = _cobs()
    rng = np.random.default_rng(21)
    # equal largest documents: equal row counts; 37 documents in a, so b's
    # columns start inside a byte and inside a dword
    A = [rand_dna(rng, int(rng.integers(1500, 5000))) for _ in range(36)] + [rand_dna(rng, 6000)]
    B = [rand_dna(rng, int(rng.integers(1500, 5000))) for _ in range(49)] + [rand_dna(rng, 6000)]
    ia, _ = _build(cobs, A, 0)
    ib, _ = _build(cobs, B, 0)
    assert ia.block(0)["rows"] == ib.block(0)["rows"]
    merged = ia.merge(ib)
    union, _ = _build(cobs, A + B, 0)
    info = merged.info()
    assert info == union.info()
    assert merged.block(0) == union.block(0)
    for x, y in zip(merged.order(), union.order()):
        assert np.array_equal(x, y)
    assert np.array_equal(merged.read(0, info["total_bytes"]), union.read(0, info["total_bytes"]))
    qs, data, off = _queries(rng, A + B)
    for x, y in zip(merged.query(data, off, k=(1, 2)), union.query(data, off, k=(1, 2))):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    # different row counts, different parameters
    ic, _ = _build(cobs, [rand_dna(rng, 9000)], 0)
    with pytest.raises(cobs.CobsError) as e:
        ia.merge(ic)
    assert e.value.status == cobs.EINVAL
    ik, _ = _build(cobs, A, 8)
    with pytest.raises(cobs.CobsError) as e:
        ia.merge(ik)
    assert e.value.status == cobs.EINVAL


def test_compact_merge_keeps_every_documents_score(tmp_path):
    cobs = _cobs()
    rng = np.random.default_rng(22)
    A = [rand_dna(rng, int(rng.integers(1200, 8000))) for _ in range(29)]
    B = [rand_dna(rng, int(rng.integers(1200, 8000))) for _ in range(21)]
    ia, da = _build(cobs, A, 8)
    ib, db = _build(cobs, B, 8)
    merged = ia.merge(ib)
    info = merged.info()
    assert info["n_docs"] == 50 and info["n_blocks"] == ia.info()["n_blocks"] + ib.info()["n_blocks"]
    oa = oracle.OracleIndex(da, kind=0, q=31, canonical=True, h=1, p=0.3, B=8, seed=7)
    ob = oracle.OracleIndex(db, kind=0, q=31, canonical=True, h=1, p=0.3, B=8, seed=7)
    qs, data, off = _queries(rng, A + B)
    sc, nt = merged.scores(data, off)
    for i, q in enumerate(qs):
        wa, la = oa.query_scores(q)
        wb, lb = ob.query_scores(q)
        assert nt[i] == la == lb
        assert np.array_equal(sc[i, :29], wa) and np.array_equal(sc[i, 29:], wb), i
    # hits come in (score desc, merged id asc) order over both parts
    for i, (ids, s, l) in enumerate(merged.query(data, off, k=(1, 2))):
        T = -(-l // 2)
        want = np.nonzero(sc[i] >= T)[0] if l else np.zeros(0, np.int64)
        want = want[np.lexsort((want, -sc[i, want].astype(np.int64)))]
        assert np.array_equal(ids, want) and np.array_equal(s, sc[i, want])
    # a merged compact index (not size-sorted across its parts) saves and loads
    path = str(tmp_path / "merged.cobs")
    merged.save(path)
    back = cobs.Index.load(path)
    sc2, nt2 = back.scores(data, off)
    assert np.array_equal(sc2, sc) and np.array_equal(nt2, nt)
