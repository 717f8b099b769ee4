"""Out-of-core queries: with the matrix in host memory and streamed through
device staging buffers group by group, every result equals the in-device one
(and therefore the oracle's, which the in-device path matches)."""
import numpy as np
import pytest

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
        _same(_results(ix, qs), before)
        _same(_results(ix, qs), before)   # staging buffers reused across batches
        for order in (cobs.ORDER_QUERIES, cobs.ORDER_SLICES):   # within each group
            ix.set_tuning(0, 0, order)
            try:
                _same(_results(ix, qs), before)
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
