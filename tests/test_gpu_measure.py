"""Measurement calls: cobs_profile counts every gather launch and its
algorithmic row bytes (sum over queries of l x h x row bytes per term, the
figure the benchmark divides by kernel time); cobs_read_bandwidth times a
plain read pass and refuses buffers it cannot read in 16-byte words."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,scale", [(3, 100), (4, 200)])
def test_profile_counts_algorithmic_row_bytes(cfg, scale):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    w = synth.CONFIGS[cfg].scaled(scale)
    d = synth.docs(w)
    kind = 0 if w.kind == "dna" else 1
    prm = cobs.make_params(kind, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    qs = synth.dna_queries(w, n=30) if w.kind == "dna" else synth.text_queries(w, d, n=30)
    info = ix.info()
    row_bytes = sum(ix.block(b)["stride"] for b in range(info["n_blocks"]))
    cobs.profile(True)
    try:
        cobs.profile_read(reset=True)
        nt = ix.query_flat(qs.bytes, qs.q_off, k=(1, 2))[0]
        nt2 = ix.query_flat(qs.bytes, qs.q_off, k=(1, 2), mode=cobs.MODE_PLAIN)[0]
        t = cobs.profile_read(reset=True)
    finally:
        cobs.profile(False)
    assert np.array_equal(nt, nt2)
    assert t["launches"] >= 2          # the batch, then one launch per query
    assert t["terms"] == 2 * int(nt.sum())
    assert t["row_bytes"] == 2 * int(nt.sum()) * w.h * row_bytes
    assert t["total_ms"] > 0


def test_read_bandwidth():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    buf = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    gbps = max(cobs.read_bandwidth(buf) for _ in range(3))
    assert 500 < gbps < 20000        # plausible for HBM, far from zero or absurd
    import ctypes
    r = ctypes.c_double()
    assert cobs.lib().cobs_read_bandwidth(ctypes.c_void_p(buf.data_ptr() + 8), 1 << 20, None,
                                          ctypes.byref(r)) == cobs.EINVAL
    assert cobs.lib().cobs_read_bandwidth(ctypes.c_void_p(buf.data_ptr()), 1000, None,
                                          ctypes.byref(r)) == cobs.EINVAL


def test_read_rows_bandwidth():
    # random 1 KiB row reads: a working set that fits the L2 reads faster than
    # one that only HBM holds; malformed buffers are refused
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    buf = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    small = cobs.read_rows_bandwidth(buf[:2 << 20], 8 << 20, cached=True)
    big = cobs.read_rows_bandwidth(buf, 8 << 20, cached=False)
    assert 500 < big < 20000 and small > big
    import ctypes
    r = ctypes.c_double()
    L = cobs.lib()
    assert L.cobs_read_rows_bandwidth(ctypes.c_void_p(buf.data_ptr() + 8), 1 << 20, 1000, 1, None,
                                      ctypes.byref(r)) == cobs.EINVAL
    assert L.cobs_read_rows_bandwidth(ctypes.c_void_p(buf.data_ptr()), 512, 1000, 1, None,
                                      ctypes.byref(r)) == cobs.EINVAL
    assert L.cobs_read_rows_bandwidth(ctypes.c_void_p(buf.data_ptr()), 1 << 20, 0, 1, None,
                                      ctypes.byref(r)) == cobs.EINVAL
