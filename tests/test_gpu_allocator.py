"""Device memory from the caller's allocator (cobs_set_allocator): an index
built, queried and served with torch's caching allocator holds its memory
there, gives the same hits as one on hipMalloc, and gives every byte back;
an allocator that fails makes the call fail with ENOMEM."""
import gc

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _cobs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    return cobs


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) and x[2] == y[2]


def test_torch_allocator_holds_and_returns_the_library_memory():
    import torch
    cobs = _cobs()
    w = synth.CONFIGS[3].scaled(100)
    d = synth.docs(w)
    prm = cobs.make_params(0, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    qs = synth.dna_queries(w, n=40)
    ref = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)     # hipMalloc
    want = ref.query(qs.bytes, qs.q_off, k=(1, 2))
    want_top = ref.query(qs.bytes, qs.q_off, k=(0, 1), topk=5, chunk=7)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    cobs.use_torch_allocator()
    try:
        ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
        assert torch.cuda.memory_allocated() - base >= ix.info()["total_bytes"]
        _same(ix.query(qs.bytes, qs.q_off, k=(1, 2)), want)
        _same(ix.query(qs.bytes, qs.q_off, k=(0, 1), topk=5, chunk=7), want_top)   # split queries
        srv = cobs.Server(ix, num_streams=2)
        tickets = [srv.submit(qs.get(i), k=(1, 2)) for i in range(qs.n)]
        for t, x in zip(tickets, want):
            got = srv.wait(t)
            assert np.array_equal(got[0], x[0]) and np.array_equal(got[1], x[1])
        srv.stop()
        # memory made before the switch goes back through hipFree
        del ref
        del ix, srv
        gc.collect()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        cobs.use_torch_allocator(False)


def test_failing_allocator_gives_enomem():
    cobs = _cobs()
    w = synth.CONFIGS[1].scaled(50)
    d = synth.docs(w)
    prm = cobs.make_params(0, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    cobs.set_allocator(lambda n: 0, lambda p: None)
    try:
        with pytest.raises(cobs.CobsError) as e:
            cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
        assert e.value.status == cobs.ENOMEM
    finally:
        cobs.set_allocator()
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)       # hipMalloc again
    assert ix.info()["n_docs"] == w.n_docs
