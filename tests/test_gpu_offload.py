"""Out-of-core queries: with the matrix in host memory and streamed through
device staging buffers group by group, every result equals the in-device one
and the oracle's (full scores, threshold hits and top-k, batched and plain),
on an index of narrow blocks and on one of 1 KiB row slices."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def built():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    w = synth.CONFIGS[3].scaled(50)
    d = synth.docs(w)
    prm = cobs.make_params(0, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    qs = synth.dna_queries(w, n=40)
    info = ix.info()
    big = max(ix.block(b)["rows"] * ix.block(b)["stride"] for b in range(info["n_blocks"]))
    return cobs, w, d, prm, ix, qs, big


def _results(ix, qs):
    return (ix.query(qs.bytes, qs.q_off, k=(1, 2)),
            ix.query(qs.bytes, qs.q_off, k=(0, 1), topk=5, chunk=7),
            ix.query(qs.bytes, qs.q_off, k=(4, 5), mode=1),
            ix.scores(qs.bytes, qs.q_off))


def _same(a, b):
    for x, y in zip(a[:3], b[:3]):
        for u, v in zip(x, y):
            assert np.array_equal(u[0], v[0]) and np.array_equal(u[1], v[1]) and u[2] == v[2]
    assert np.array_equal(a[3][0], b[3][0]) and np.array_equal(a[3][1], b[3][1])


def test_offloaded_results_equal_device_resident(built):
    cobs, w, d, prm, ix, qs, big = built
    info = ix.info()
    assert info["n_blocks"] >= 4 and not info["host_resident"]
    before = _results(ix, qs)
    matrix = ix.read(0, info["total_bytes"])
    # staging buffers that hold one or two blocks: several groups per batch
    ix.offload(2 * ((big + 255) // 256 * 256))
    try:
        info2 = ix.info()
        assert info2["host_resident"] and info2["n_groups"] >= 2
        assert info2["stage_bytes"] >= big
        assert np.array_equal(ix.read(0, info["total_bytes"]), matrix)
        _same(_results(ix, qs), before)   # automatic choice of host reads
        for mode in (cobs.HOST_READS_STREAM, cobs.HOST_READS_IN_PLACE):
            for order in (cobs.ORDER_AUTO, cobs.ORDER_QUERIES, cobs.ORDER_SLICES):
                ix.set_tuning(0, 0, order, mode)
                try:
                    _same(_results(ix, qs), before)
                    _same(_results(ix, qs), before)   # staging buffers reused across batches
                finally:
                    ix.set_tuning(0, 0)
        srv = cobs.Server(ix, num_streams=3)
        tickets = [srv.submit(qs.get(i), k=(1, 2)) for i in range(qs.n)]
        served = [srv.wait(t) for t in tickets]
        srv.stop()
        for s, b in zip(served, before[0]):
            assert np.array_equal(s[0], b[0]) and np.array_equal(s[1], b[1])
        with pytest.raises(cobs.CobsError) as e:
            ix.offload(1 << 30)
        assert e.value.status == cobs.ESTATE
    finally:
        ix.onload()
    assert not ix.info()["host_resident"]
    assert np.array_equal(ix.read(0, info["total_bytes"]), matrix)
    _same(_results(ix, qs), before)


def test_offload_budget_must_hold_the_largest_block(built):
    cobs, w, d, prm, ix, qs, big = built
    with pytest.raises(cobs.CobsError) as e:
        ix.offload(2 * big - 1024)
    assert e.value.status == cobs.EBUDGET
    assert not ix.info()["host_resident"]
    with pytest.raises(cobs.CobsError) as e:
        ix.onload()
    assert e.value.status == cobs.ESTATE
    # a budget for the whole matrix: one group
    ix.offload(2 * ix.info()["total_bytes"] + 4096)
    try:
        assert ix.info()["n_groups"] == 1
        got = ix.query(qs.bytes, qs.q_off, k=(1, 2))
    finally:
        ix.onload()
    want = ix.query(qs.bytes, qs.q_off, k=(1, 2))
    for u, v in zip(got, want):
        assert np.array_equal(u[0], v[0]) and np.array_equal(u[1], v[1])


def _rand(rng, n):
    return rng.choice(np.frombuffer(b"ACGT", np.uint8), n).tobytes()


def _wide_collection():
    # 20,000 short documents in blocks of 8,192: two blocks of 1 KiB row
    # slices and a narrow last one
    rng = np.random.default_rng(4242)
    docs = [[_rand(rng, int(rng.integers(40, 400)))] for _ in range(20000)]
    qs = [b"", _rand(rng, 3000)]
    for j in range(30):
        s = docs[int(rng.integers(0, len(docs)))][0]
        qs.append(s[int(rng.integers(0, len(s) - 31)):])
        qs.append(_rand(rng, int(rng.integers(31, 400))))
    return oracle.Docs.from_lists(docs), qs, 8192, 0xC0FFEE


def _narrow_collection():
    w = synth.CONFIGS[3].scaled(50)      # 2,000 documents, blocks of 163
    d = synth.docs(w)
    qs = synth.dna_queries(w, n=40)
    return oracle.Docs(d.bytes, d.str_off, d.doc_str), [qs.get(i) for i in range(qs.n)], w.B, w.hash_seed


@pytest.mark.parametrize("which", ["narrow", "wide"])
def test_offloaded_results_equal_oracle(which):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    d, qs, B, seed = _narrow_collection() if which == "narrow" else _wide_collection()
    prm = cobs.make_params(0, 31, True, 1, 0.3, B, seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    oix = oracle.OracleIndex(d, kind=oracle.DNA, q=31, canonical=True, h=1, p=0.3, B=B, seed=seed)
    info = ix.info()
    strides = [ix.block(b)["stride"] for b in range(info["n_blocks"])]
    assert (max(strides) >= 1024) == (which == "wide")
    big = max(ix.block(b)["rows"] * ix.block(b)["stride"] for b in range(info["n_blocks"]))
    off = np.zeros(len(qs) + 1, np.uint64)
    np.cumsum([len(x) for x in qs], out=off[1:])
    data = np.frombuffer(b"".join(qs), np.uint8)
    want = [oix.query_scores(x) for x in qs]
    # staging buffers of about one block each: several groups per batch;
    # the matrix streamed group by group, then read in place
    ix.offload(2 * ((big + 255) // 256 * 256))
    try:
        assert ix.info()["host_resident"] and ix.info()["n_groups"] >= 2
        for host_reads in (cobs.HOST_READS_STREAM, cobs.HOST_READS_IN_PLACE):
            ix.set_tuning(host_reads=host_reads)
            sc, nt = ix.scores(data, off)
            for j in range(len(qs)):
                assert nt[j] == want[j][1] and np.array_equal(sc[j], want[j][0]), (host_reads, j)
            # the last two: early exit of threshold queries (same results)
            for k, topk, mode, chunk, prune in (((4, 5), 0, 0, 0, 0), ((1, 2), 0, 1, 0, 0),
                                                ((0, 1), 5, 0, 7, 0), ((4, 5), 0, 0, 0, 1),
                                                ((1, 2), 3, 1, 0, 1)):
                ix.set_tuning(host_reads=host_reads, prune=prune)
                got = ix.query(data, off, k=k, topk=topk, mode=mode, chunk=chunk)
                for j, x in enumerate(qs):
                    ids, scores, l = oix.query(x, k[0], k[1], topk)
                    assert got[j][2] == l and np.array_equal(got[j][0], ids), (host_reads, j, k)
                    assert np.array_equal(got[j][1], scores), (host_reads, j, k)
    finally:
        ix.set_tuning()
        ix.onload()
