"""The allocation-free entry point (cobs_query_scores_noalloc) against the
allocating one it varies (cobs_query_scores) and the oracle: full score
vectors and distinct-term counts, bit-exact, on two calls in a row on one
device (the second with a smaller batch, so that it runs over what the first
left in the shared scratch array), then a batch too large for the scratch
array, refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    torch.cuda.set_device(0)
    return torch, cobs


def _noalloc(torch, ix, data, off, nd):
    n = len(off) - 1
    d = torch.from_numpy(data.copy()).to("cuda")
    sc = torch.full((n * nd,), 0x7FFFFFFF, dtype=torch.int32, device="cuda")   # overwritten
    nt = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    ix.scores_noalloc(d, off, sc, nt)
    torch.cuda.synchronize()
    return (sc.cpu().numpy().view(np.uint32).reshape(n, nd), nt.cpu().numpy().view(np.uint32))


def test_noalloc_scores_equal_allocating_entry_point_twice():
    torch, cobs = _setup()
    # 400 documents in blocks of 32 (13 blocks), queries long enough to be
    # split into several work items (tickets, score buffers), two longer than
    # an LDS set (their windows deduplicated in hash partitions), plus an
    # empty query and one shorter than q
    w = synth.CONFIGS[3].scaled(250, "noalloc")
    d = synth.docs(w)
    prm = cobs.make_params(cobs.DNA, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    nd = ix.info()["n_docs"]
    oix = oracle.OracleIndex(oracle.Docs(d.bytes, d.str_off, d.doc_str), kind=oracle.DNA, q=w.q,
                             canonical=w.canonical, h=w.h, p=w.p, B=w.B, seed=w.hash_seed)
    qs = synth.dna_queries(w, n=40)
    rng = np.random.default_rng(77)
    longs = [rng.choice(np.frombuffer(b"ACGT", np.uint8), n).tobytes() for n in (20000, 30000)]
    strings = [qs.get(i) for i in range(qs.n)] + longs + [b"", b"ACGT" * 5]
    for call, subset in enumerate([strings, strings[3:11] + strings[-2:]]):
        data = np.frombuffer(b"".join(subset), np.uint8).copy()
        off = np.zeros(len(subset) + 1, np.uint64)
        off[1:] = np.cumsum([len(s) for s in subset])
        print(f"noalloc call {call + 1}: {len(subset)} queries, {data.size} bytes", flush=True)
        want_sc, want_nt = ix.scores(data, off)
        got_sc, got_nt = _noalloc(torch, ix, data, off, nd)
        assert np.array_equal(got_nt, want_nt)
        assert np.array_equal(got_sc, want_sc)
        for i, s in enumerate(subset):
            osc, ol = oix.query_scores(s)
            assert ol == got_nt[i]
            assert np.array_equal(got_sc[i], osc), i


def test_noalloc_refuses_a_batch_beyond_its_scratch_array():
    torch, cobs = _setup()
    w = synth.CONFIGS[3].scaled(2000, "noalloc-small")
    d = synth.docs(w)
    prm = cobs.make_params(cobs.DNA, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    nd = ix.info()["n_docs"]
    n_bytes = 3 << 20                     # one query of about 3 M windows: > 64 MiB of buffers
    data = torch.zeros(n_bytes, dtype=torch.uint8, device="cuda")
    off = np.array([0, n_bytes], np.uint64)
    sc = torch.zeros(nd, dtype=torch.int32, device="cuda")
    with pytest.raises(cobs.CobsError) as e:
        ix.scores_noalloc(data, off, sc)
    assert e.value.status == cobs.EBUDGET
    # NULL outputs are refused too
    assert cobs.lib().cobs_query_scores_noalloc(ix._h, ctypes.c_void_p(data.data_ptr()),
                                                off.ctypes.data_as(ctypes.c_void_p), 1, None,
                                                None, None) == cobs.EINVAL
