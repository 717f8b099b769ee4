"""A seeded sweep over the parameter space on tiny collections: q from 1 to
its maximum, canonical or not, h from 1 to 8, p from 0.01 to 0.9, classic and
compact with B from 1 upward, documents that are empty, shorter than q, made
of several strings, with lower-case and non-ACGT bytes.  In every case the
index (distinct counts, order, block table, matrix bytes) and every query's
full score vector and hits equal the oracle's."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(20261203)
    out = []
    for i in range(24):
        kind = 1 if i % 3 == 0 else 0
        q = int(rng.integers(1, 9)) if kind else int(rng.integers(1, 32))
        canonical = bool(rng.integers(0, 2)) if not kind else False
        h = int(rng.integers(1, 9))
        p = float(rng.choice([0.01, 0.1, 0.3, 0.5, 0.9]))
        B = int(rng.choice([0, 1, 3, 8, 17, 64]))
        out.append((i, kind, q, canonical, h, p, B))
    # the extremes of each range
    out += [(100, 0, 31, True, 8, 0.01, 1), (101, 0, 1, False, 1, 0.9, 0),
            (102, 1, 8, False, 8, 0.5, 2), (103, 1, 1, False, 3, 0.3, 5),
            (104, 0, 31, False, 1, 0.3, 0), (105, 0, 2, True, 2, 0.1, 7)]
    return out


def _string(rng, kind, n):
    if kind:
        return rng.integers(0, 256, n, dtype=np.uint8).tobytes()
    # mostly ACGT, some lower case, a few N
    alphabet = np.frombuffer(b"ACGTACGTACGTACGTacgtN", np.uint8)
    return rng.choice(alphabet, n).tobytes()


def _collection(rng, kind, q):
    docs = []
    for _ in range(int(rng.integers(1, 41))):
        strings = [_string(rng, kind, int(rng.integers(0, 5 * q + 60)))
                   for _ in range(int(rng.integers(0, 4)))]
        docs.append(strings)
    return docs


def _queries(rng, kind, q, docs):
    qs = [b"", _string(rng, kind, max(q - 1, 0)), _string(rng, kind, 3 * q + 40)]
    for d in docs[:6]:
        for s in d:
            if len(s) >= q:
                a = int(rng.integers(0, len(s) - q + 1))
                qs.append(s[a:a + int(rng.integers(q, len(s) - a + 1))])
                break
    off = np.zeros(len(qs) + 1, np.uint64)
    np.cumsum([len(x) for x in qs], out=off[1:])
    data = np.frombuffer(b"".join(qs), np.uint8) if off[-1] else np.zeros(0, np.uint8)
    return qs, data, off


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"c{c[0]}-{'bytes' if c[1] else 'dna'}-q{c[2]}-h{c[4]}-B{c[6]}")
def test_parameter_sweep_matches_oracle(case):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    i, kind, q, canonical, h, p, B = case
    rng = np.random.default_rng(1000 + i)
    docs = _collection(rng, kind, q)
    d = oracle.Docs.from_lists(docs)
    seed = 0x5EED + i
    prm = cobs.make_params(kind, q, canonical, h, p, B, seed)
    gix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    oix = oracle.OracleIndex(d, kind=kind, q=q, canonical=canonical, h=h, p=p, B=B, seed=seed)
    order, nterms = gix.order()
    assert np.array_equal(nterms, oix.n_terms())
    assert np.array_equal(order, oix.order())
    assert gix.info()["n_blocks"] == oix.n_blocks
    omat = oix.matrix()
    for b in range(oix.n_blocks):
        gb, ob = gix.block(b), oix.block(b)
        for key in ("first", "docs", "rows", "stride"):
            assert gb[key] == ob[key], (b, key)
        n = ob["rows"] * ob["stride"]
        assert np.array_equal(gix.read(gb["offset"], n), omat[ob["offset"]:ob["offset"] + n]), b
    qs, data, off = _queries(rng, kind, q, docs)
    sc, nt = gix.scores(data, off)
    for j, x in enumerate(qs):
        want, wl = oix.query_scores(x)
        assert nt[j] == wl and np.array_equal(sc[j], want), j
    for k, topk in (((1, 2), 0), ((0, 1), 3), ((9, 10), 0)):
        got = gix.query(data, off, k=k, topk=topk)
        for j, x in enumerate(qs):
            ids, scores, l = oix.query(x, k[0], k[1], topk)
            assert got[j][2] == l and np.array_equal(got[j][0], ids), (j, k, topk)
            assert np.array_equal(got[j][1], scores), (j, k, topk)


@pytest.mark.parametrize("B", [0, 2])
def test_collection_without_terms(B):
    # no document has a window (no strings, empty strings, strings shorter
    # than q): every block gets one zero row and every score is 0
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    d = oracle.Docs.from_lists([[], [b"ACGT"], [b""], [], [b"ACGTACGTAC", b"GG"]])
    prm = cobs.make_params(0, 31, True, 2, 0.3, B, 9)
    gix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    oix = oracle.OracleIndex(d, kind=0, q=31, canonical=True, h=2, p=0.3, B=B, seed=9)
    order, nterms = gix.order()
    assert np.array_equal(nterms, oix.n_terms()) and not nterms.any()
    assert np.array_equal(order, oix.order())
    for b in range(oix.n_blocks):
        gb, ob = gix.block(b), oix.block(b)
        assert (gb["rows"], gb["stride"]) == (ob["rows"], ob["stride"]) == (1, 128)
        assert not gix.read(gb["offset"], 128).any()
    data = np.frombuffer(b"ACGT" * 20 + b"TTTTGGGGCCCCAAAATTTTGGGGCCCCAAAA", np.uint8)
    off = np.array([0, 80, 112], np.uint64)
    for x, (q0, q1) in zip(gix.query(data, off, k=(0, 1)), ((0, 80), (80, 112))):
        ids, sc, l = oix.query(data[q0:q1].tobytes(), 0, 1, 0)
        assert x[2] == l and np.array_equal(x[0], ids) and np.array_equal(x[1], sc)


def _wide_cases():
    # (kind, q, canonical, h, p, B, documents): blocks wider than 4,096
    # documents, so the gather runs its unpacked instantiations (one term per
    # 1 KiB load, h rows ANDed per term) for every h from 2 to 8
    return [(0, 31, True, 2, 0.3, 0, 4600), (1, 8, False, 3, 0.1, 8192, 9000),
            (0, 21, False, 4, 0.2, 0, 5000), (1, 5, False, 5, 0.05, 0, 4200),
            (0, 31, True, 6, 0.3, 5000, 9100), (1, 8, False, 7, 0.5, 0, 4400),
            (0, 15, True, 8, 0.01, 8192, 8500)]


@pytest.mark.parametrize("case", _wide_cases(), ids=lambda c: f"{'bytes' if c[0] else 'dna'}-h{c[3]}-B{c[5]}-D{c[6]}")
def test_wide_blocks_every_h_match_oracle(case):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    kind, q, canonical, h, p, B, n_docs = case
    rng = np.random.default_rng(7000 + 10 * h + kind)
    docs = [[_string(rng, kind, int(rng.integers(q, q + 150)))] for _ in range(n_docs)]
    d = oracle.Docs.from_lists(docs)
    seed = 0xB10C + h
    prm = cobs.make_params(kind, q, canonical, h, p, B, seed)
    gix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    oix = oracle.OracleIndex(d, kind=kind, q=q, canonical=canonical, h=h, p=p, B=B, seed=seed)
    # a slice wider than 512 bytes: the index is gathered one term per load
    info = gix.info()
    assert max(gix.block(b)["stride"] for b in range(info["n_blocks"])) > 512
    # queries: planted substrings, random strings, and one long enough to be
    # split into several work items
    qs = [b"", _string(rng, kind, 4000)]
    for j in range(24):
        s = docs[int(rng.integers(0, n_docs))][0]
        a = int(rng.integers(0, len(s) - q + 1))
        qs.append(s[a:])
        qs.append(_string(rng, kind, int(rng.integers(q, 200))))
    off = np.zeros(len(qs) + 1, np.uint64)
    np.cumsum([len(x) for x in qs], out=off[1:])
    data = np.frombuffer(b"".join(qs), np.uint8)
    want = [oix.query_scores(x) for x in qs]
    for unroll in (2, 4):
        gix.set_tuning(unroll, 0)
        sc, nt = gix.scores(data, off)
        for j in range(len(qs)):
            assert nt[j] == want[j][1] and np.array_equal(sc[j], want[j][0]), (unroll, j)
        for k, topk, mode in (((4, 5), 0, 0), ((1, 2), 0, 1), ((0, 1), 5, 0)):
            got = gix.query(data, off, k=k, topk=topk, mode=mode)
            for j, x in enumerate(qs):
                ids, scores, l = oix.query(x, k[0], k[1], topk)
                assert got[j][2] == l and np.array_equal(got[j][0], ids), (unroll, j, k)
                assert np.array_equal(got[j][1], scores), (unroll, j, k)
    gix.set_tuning(0, 0)
