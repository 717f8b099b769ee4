"""Continuous-batching server: every request's result equals the batch path's
(and the oracle's), alone or in a mix; admission by score memory."""
import threading

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    w = synth.CONFIGS[3].scaled(200)
    d = synth.docs(w)
    prm = cobs.make_params(0, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    from dataclasses import replace
    wq = replace(w, q_len=("loguniform", 31, 20_000))
    qs = synth.dna_queries(wq, n=60)
    oix = oracle.OracleIndex(oracle.Docs(d.bytes, d.str_off, d.doc_str), kind=0, q=w.q,
                             canonical=w.canonical, h=w.h, p=w.p, B=w.B, seed=w.hash_seed)
    return cobs, ix, qs, oix


def test_served_results_equal_batch_and_oracle(served):
    cobs, ix, qs, oix = served
    batch = ix.query(qs.bytes, qs.q_off, k=(1, 2))
    srv = cobs.Server(ix, num_streams=3, max_batch_queries=16)
    tickets = [srv.submit(qs.get(i), k=(1, 2)) for i in range(qs.n)]
    got = [srv.wait(t) for t in tickets]
    st = srv.stop()
    assert st["completed"] == qs.n and st["batches"] >= 1
    for i, (ids, sc, l, lat) in enumerate(got):
        assert np.array_equal(ids, batch[i][0]) and np.array_equal(sc, batch[i][1]), i
        w_ids, w_sc, wl = oix.query(qs.get(i), 1, 2, 0)
        assert l == wl and np.array_equal(ids, w_ids) and np.array_equal(sc, w_sc), i
        assert lat > 0


def test_served_with_early_exit_equal_oracle(served):
    # the server over an index with early exit on (batches of queries up to
    # 20 kbp, split over chunks: two pruning launches): the oracle's hits
    cobs, ix, qs, oix = served
    ix.set_tuning(prune=cobs.PRUNE_ON)
    try:
        srv = cobs.Server(ix, num_streams=3, max_batch_queries=16)
        tickets = [srv.submit(qs.get(i), k=(4, 5), topk=i % 3) for i in range(qs.n)]
        got = [srv.wait(t) for t in tickets]
        srv.stop()
    finally:
        ix.set_tuning()
    for i, (ids, sc, l, lat) in enumerate(got):
        w_ids, w_sc, wl = oix.query(qs.get(i), 4, 5, i % 3)
        assert l == wl and np.array_equal(ids, w_ids) and np.array_equal(sc, w_sc), i


def test_same_result_alone_and_in_a_mix(served):
    cobs, ix, qs, oix = served
    x = qs.get(0)
    srv = cobs.Server(ix, num_streams=2)
    alone = srv.wait(srv.submit(x, k=(4, 5), topk=3))
    # the same request while others (different options too) arrive around it
    stop = threading.Event()

    def noise():
        j = 1
        while not stop.is_set():
            t = srv.submit(qs.get(j % qs.n), k=(1, 2) if j % 2 else (4, 5), topk=j % 3)
            srv.wait(t)
            j += 1

    ths = [threading.Thread(target=noise) for _ in range(4)]
    for t in ths:
        t.start()
    mixed = [srv.wait(srv.submit(x, k=(4, 5), topk=3)) for _ in range(10)]
    stop.set()
    for t in ths:
        t.join()
    srv.stop()
    for m in mixed:
        assert np.array_equal(m[0], alone[0]) and np.array_equal(m[1], alone[1]) and m[2] == alone[2]
    w_ids, w_sc, wl = oix.query(x, 4, 5, 3)
    assert np.array_equal(alone[0], w_ids) and np.array_equal(alone[1], w_sc)


def test_admission_by_score_memory(served):
    cobs, ix, qs, oix = served
    info = ix.info()
    per_query = info["score_bytes"]
    # 4 bytes per document, each block's 8192-document slices rounded up to
    # whole 128-document lanes
    want = 0
    for b in range(info["n_blocks"]):
        docs = ix.block(b)["docs"]
        for s0 in range(0, docs, 8192):
            want += 4 * 128 * (-(-min(8192, docs - s0) // 128))
    assert per_query == want >= 4 * info["n_docs"]
    with pytest.raises(cobs.CobsError) as e:
        srv = cobs.Server(ix, budget_bytes=per_query - 1)
        try:
            srv.submit(qs.get(1))
        finally:
            srv.stop()
    assert e.value.status == cobs.EBUDGET
    # room for two requests at a time: the rest wait for admission, all finish
    srv = cobs.Server(ix, budget_bytes=2 * per_query, num_streams=2)
    tickets = [srv.submit(qs.get(i), k=(1, 2)) for i in range(12)]
    res = [srv.wait(t) for t in tickets]
    st = srv.stop()
    assert st["completed"] == 12 and st["rejected"] == 0
    batch = ix.query(qs.bytes[: int(qs.q_off[12])], qs.q_off[:13], k=(1, 2))
    for a, b in zip(res, batch):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # one request admitted at a time (max_inflight): every batch holds exactly one
    srv = cobs.Server(ix, num_streams=2, max_inflight=1)
    tickets = [srv.submit(qs.get(i), k=(1, 2)) for i in range(12)]
    res = [srv.wait(t) for t in tickets]
    st = srv.stop()
    assert st["completed"] == 12 and st["batches"] == 12
    for a, b in zip(res, batch):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_open_loop_replay_and_stats(served):
    cobs, ix, qs, oix = served
    arrivals = synth.arrivals(11, qs.n, 2000.0)
    srv = cobs.Server(ix, num_streams=2)
    lat, nh = srv.replay(qs.bytes, qs.q_off, arrivals, k=(1, 2))
    st = srv.stop()
    assert st["completed"] == qs.n
    assert np.all(lat > 0)
    assert st["p50_ns"] <= st["p99_ns"] <= st["max_ns"]
    batch = ix.query(qs.bytes, qs.q_off, k=(1, 2))
    assert [len(b[0]) for b in batch] == list(nh)


def test_stop_drains_pending_requests(served):
    cobs, ix, qs, oix = served
    srv = cobs.Server(ix, num_streams=1, max_batch_queries=4)
    for i in range(20):
        srv.submit(qs.get(i % qs.n))
    st = srv.stop()
    assert st["completed"] == 20 and st["submitted"] == 20
