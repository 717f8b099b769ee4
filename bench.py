#!/usr/bin/env python3
"""Benchmark of the COBS query hot path on one MI355X.

Workload (default): the compact 100,000-document index -- random ACGT
documents with distinct 31-mer counts log-normal (median 1M, sigma 0.7,
capped at 8M), size-sorted blocks of 8,192, h = 1, p = 0.3 -- queried with
10,000 DNA queries of log-uniform length in [100, 10,000] bp (half planted
substrings with 1% substitutions), threshold K = 0.8.  The index is built on
the device (documents generated straight into HBM, two passes through the
streaming builder) and stays resident; the query bytes are resident in HBM
when the timed region starts.

One step = one cobs_query_batch over the whole query set: term extraction,
dedup + hashing, planning, the persistent gather/AND/ADD/threshold kernel,
and the ordering of the hits, results copied back to the host.

Prints ONE JSON line (rank 0) with the k-mer lookup rate, the roofline of
the gather kernel (HBM-bound), and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(msg: str) -> None:
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4])
    ap.add_argument("--scale", type=int, default=1, help="divide the workload by this factor")
    ap.add_argument("--queries", type=int, default=0, help="override the query count")
    ap.add_argument("--plain-queries", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chunk-gb", type=float, default=8.0,
                    help="device bytes of documents generated per build run")
    ap.add_argument("--serve-rates", type=str, default="1000,2700,7100,18800,50000",
                    help="Poisson arrival rates (q/s) of the serving measurement; '' skips it")
    ap.add_argument("--serve-pool", type=int, default=1000)
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-max", type=int, default=8000)
    ap.add_argument("--serve-streams", type=int, default=4, help="batches in flight in the server")
    ap.add_argument("--tuning", type=str, default="",
                    help="'unroll,chunk[,order]' launch shape instead of autotuning")
    ap.add_argument("--offload-gb", type=float, default=30.0,
                    help="last: move the matrix to host memory and time streamed batches "
                         "with this device budget (GB) for the staging buffers; 0 skips it")
    ap.add_argument("--calib-copy-gb", type=float, default=0.0,
                    help="run one plain device copy of this size (counter calibration)")
    return ap.parse_args()


def build_index_dna(cobs, synth, torch, w, chunk_bytes):
    """Streamed two-pass build: documents generated on the device per run."""
    import numpy as np
    lens = synth.doc_lengths(w)
    n = w.n_docs
    runs, a, acc = [], 0, 0
    for d in range(n):
        L = int(lens[d])
        if d > a and acc + L > chunk_bytes:
            runs.append((a, d))
            a, acc = d, 0
        acc += L
    runs.append((a, n))
    maxrun = max(int(lens[a:b].sum()) for a, b in runs)
    buf = torch.empty(maxrun + 64, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def gen(pass_no):
        t0 = time.time()
        for k, (a, b) in enumerate(runs):
            off = np.zeros(b - a + 1, np.uint64)
            np.cumsum(lens[a:b], out=off[1:])
            doff = torch.from_numpy(off.view(np.int64)).to("cuda")
            synth.dna_docs_device(w, a, b - a, buf.data_ptr(), doff.data_ptr(), stream.cuda_stream)
            yield a, buf, off, np.arange(b - a + 1, dtype=np.uint64)
            if k % 8 == 0 or k == len(runs) - 1:
                log(f"build pass {pass_no}: run {k + 1}/{len(runs)} docs {b} "
                    f"({time.time() - t0:.1f}s)")

    prm = cobs.make_params(cobs.DNA, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    ix = cobs.Index.build_streamed(prm, n, gen)
    del buf
    return ix


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "gather_compact100k_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1905_09624_amd", "csrc", "gather.hip")


def committed_traffic(workload: str):
    """HBM bytes per gather launch from the committed rocprofv3 --pmc summary
    (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or None when
    the kernel source changed since the counters were taken or the summary
    covers another workload."""
    import hashlib
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    fields = {}
    for line in open(TRAFFIC_SUMMARY):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            fields[k.strip()] = v.strip().strip("`")
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if fields.get("gather.hip sha256") != src or fields.get("workload") != workload:
        return None
    try:
        return int(fields["HBM bytes per gather launch"])
    except (KeyError, ValueError):
        return None


def serve_measure(cobs, synth, torch, ix, rates, pool_n, per_rate_s, max_req, plain_n, streams,
                  set_launch=None, set_prune=None):
    """Served latency and throughput on the resident index: Poisson arrivals at
    each rate (open loop, native submitter), query lengths log-uniform in
    [31, 10^6] bp, half planted; beside it the plain path (one query per
    launch, back to back) and one batch of the whole pool.  With set_prune,
    the plain path and the server again with early exit of threshold queries
    (same results)."""
    import numpy as np
    w5 = synth.CONFIGS[5]
    t0 = time.time()
    pool = synth.dna_queries(w5, n=pool_n)
    log(f"serving pool: {pool_n} queries, {pool.bytes.size / 1e6:.1f} MB ({time.time() - t0:.1f}s)")
    k = w5.k
    out = {"workload": "serve-100k: compact-100k index resident, queries log-uniform "
                       "[31, 1e6] bp, 50% planted, Poisson arrivals", "streams": streams,
           "rates": []}
    # plain path: closed loop, one query per launch
    sub = pool.subset(range(min(plain_n, pool_n)))

    def closed_loop():
        lat = []
        nt_total = 0
        for i in range(sub.n):
            q = np.frombuffer(sub.get(i), np.uint8)
            off = np.array([0, q.size], np.uint64)
            t1 = time.perf_counter()
            nt = ix.query_flat(q, off, k=k, mode=cobs.MODE_PLAIN)[0]
            lat.append(time.perf_counter() - t1)
            nt_total += int(nt.sum())
        lat = np.array(lat)
        return {"queries_per_s": sub.n / lat.sum(), "lookups_per_s": nt_total / lat.sum(),
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "queries": sub.n}

    plain = closed_loop()
    out["plain_path"] = plain
    log(f"serving plain path: {plain}")
    # the whole pool as one batch (host bytes, as the server receives them)
    t1 = time.perf_counter()
    nt = ix.query_flat(pool.bytes, pool.q_off, k=k)[0]
    bt = time.perf_counter() - t1
    out["one_batch"] = {"queries_per_s": pool_n / bt, "lookups_per_s": float(nt.sum()) / bt,
                        "seconds": bt}
    def replay(n, rate, **opts):
        idx = np.arange(n) % pool_n
        q = pool.subset(idx) if n != pool_n else pool
        arr = synth.arrivals(0x5E7E + int(rate), n, float(rate))
        srv = cobs.Server(ix, **opts)
        srv.replay(q.bytes, q.q_off, arr, k=k)
        st = srv.stop()
        return {"requests": n, "completed": int(st["completed"]),
                "batches": int(st["batches"]), "p50_ms": st["p50_ns"] / 1e6,
                "p99_ms": st["p99_ns"] / 1e6, "max_ms": st["max_ns"] / 1e6,
                "queries_per_s": st["queries_per_s"], "lookups_per_s": st["lookups_per_s"]}

    for rate in rates:
        n = int(min(max_req, max(rate * per_rate_s, 200)))
        rec = {"rate_qps": rate, **replay(n, rate, num_streams=streams)}
        rec["vs_plain_throughput"] = rec["queries_per_s"] / plain["queries_per_s"]
        # the plain path served: one query per launch, first come first served;
        # beyond its capacity the queue only grows, so fewer requests are sent
        n_p = int(min(n, max(200, 2 * plain["queries_per_s"])))
        rec["plain_served"] = replay(n_p, rate, num_streams=1, max_batch_queries=1)
        if set_launch is not None and rate == rates[0]:
            # the lowest rate again with every kernel launched on the stream
            # (single-query batches are otherwise replayed graphs)
            set_launch(cobs.LAUNCH_DIRECT)
            rec["direct_launches"] = replay(n, rate, num_streams=streams)
            rec["plain_served_direct_launches"] = replay(n_p, rate, num_streams=1, max_batch_queries=1)
            set_launch(cobs.LAUNCH_AUTO)
        out["rates"].append(rec)
        log(f"serving at {rate} q/s: {rec}")
    if set_prune is not None:
        set_prune(True)
        pp = closed_loop()
        out["pruned"] = {"plain_path": pp, "rates": []}
        log(f"serving plain path, pruned: {pp}")
        for rate in rates:
            n = int(min(max_req, max(rate * per_rate_s, 200)))
            rec = {"rate_qps": rate, **replay(n, rate, num_streams=streams)}
            rec["vs_plain_throughput"] = rec["queries_per_s"] / plain["queries_per_s"]
            rec["vs_plain_pruned_throughput"] = rec["queries_per_s"] / pp["queries_per_s"]
            out["pruned"]["rates"].append(rec)
            log(f"serving at {rate} q/s, pruned: {rec}")
        set_prune(False)
    return out


def _timed_lookups(parts, queries, seconds, threads):
    """Score queries (cycled) against every oracle sub-index in `parts` for
    about `seconds` on `threads` threads: (distinct terms scored, wall s)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(q):
        l = 0
        for ix in parts:
            l = ix.query_scores(q)[1]
        return l

    done_l, i = 0, 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        while time.perf_counter() - t0 < seconds:
            batch = [queries[j % len(queries)] for j in range(i, i + 2 * threads)]
            done_l += sum(ex.map(one, batch))
            i += len(batch)
    return done_l, time.perf_counter() - t0


def cpu_baseline_block(w, synth, oracle, qs, order, n_terms, budget_s, threads):
    """The CPU oracle on the compact index's first block, whole: its 8,192
    documents (the smallest, in the compact order) as 16 classic oracle
    sub-indexes of 512 documents built in parallel, each with the block's
    largest document added so that every sub-index has the block's row count
    m_0 (the index build is not timed).  Queries of the query set (cycled)
    are scored against all 16 sub-indexes.  Every call of the oracle's query
    costs a per-lookup part (terms, sort, hashing) plus a part per document,
    so the oracle's rate on one index of all 100,000 documents follows from
    the per-lookup cost a (timed on the block's largest document alone) and
    the per-document cost b from the whole block on one thread: one lookup
    costs a + b * 100,000.  The same model predicts the half block (8
    sub-indexes), which is timed too: the difference is the model's error on
    this block.  The rate with `threads` threads is the one-thread rate times
    the speed-up measured over the block."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    B = w.B
    members = [int(x) for x in order[:B]]
    big = members[-1]
    rows = oracle.filter_rows(int(n_terms[big]), w.h, w.p)
    groups = [members[g * 512:(g + 1) * 512] for g in range(B // 512)]
    lens = synth.doc_lengths(w)

    def doc(d):
        out = np.empty(int(lens[d]), np.uint8)
        synth.lib().synth_doc_bases(w.seed, d, 0, int(lens[d]), synth._p(out))
        return out.tobytes()

    def build(ids):
        ix = oracle.OracleIndex(oracle.Docs.from_lists([doc(d) for d in ids]), kind=oracle.DNA,
                                q=w.q, canonical=w.canonical, h=w.h, p=w.p, B=0,
                                seed=w.hash_seed)
        assert ix.block(0)["rows"] == rows
        return ix, len(ids)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(min(16, threads)) as ex:
        built = list(ex.map(build, [g if big in g else g + [big] for g in groups] + [[big]]))
    build_s = time.perf_counter() - t0
    alone = built.pop()[0]
    parts = [b[0] for b in built]
    cols = sum(b[1] for b in built)
    half = len(parts) // 2
    half_cols = sum(b[1] for b in built[:half])
    queries = [qs.get(i) for i in range(qs.n)]
    l_a, t_a = _timed_lookups([alone], queries, budget_s / 6, 1)
    l_1, t_1 = _timed_lookups(parts, queries, budget_s / 3, 1)
    l_h, t_h = _timed_lookups(parts[:half], queries, budget_s / 6, 1)
    l_n, t_n = _timed_lookups(parts, queries, budget_s / 3, threads)
    a = t_a / l_a                                   # s per lookup, one call on one document
    b = (t_1 / l_1 - len(parts) * a) / (cols - len(parts))
    pred_half = half * a + (half_cols - half) * b
    err = pred_half / (t_h / l_h) - 1.0
    rate_1 = 1.0 / (a + b * (w.n_docs - 1))
    speedup = (l_n / t_n) / (l_1 / t_1)
    del parts, built, alone
    return {"value": rate_1 * speedup, "unit": "lookups/s", "cores": threads, "kind": "oracle",
            "value_1_thread": rate_1,
            "sample": f"block 0 of the compact plan, whole: its {B} smallest documents as "
                      f"{len(groups)} classic oracle sub-indexes of 512 (plus the block's largest "
                      f"document: m_0 = {rows} rows each, {cols} columns), built in parallel in "
                      f"{build_s:.0f}s (not timed); queries of the set cycled: {l_1 / t_1:.4g} "
                      f"lookups/s over the block on one thread ({t_1:.0f}s), {l_n / t_n:.4g} on "
                      f"{threads} ({t_n:.0f}s, speed-up {speedup:.2f}); per lookup a = "
                      f"{a * 1e9:.0f} ns (the largest document alone) plus b = {b * 1e9:.3f} ns per "
                      f"document, so {1e9 * (a + b * (w.n_docs - 1)):.0f} ns per lookup over "
                      f"{w.n_docs} documents; the same model predicts the half block "
                      f"({half} sub-indexes) {err:+.1%} off its measured time",
            "block_lookups_per_s_1_thread": l_1 / t_1, "block_lookups_per_s": l_n / t_n,
            "ns_per_lookup": a * 1e9, "ns_per_lookup_document": b * 1e9,
            "model_error_half_block": err, "build_s": build_s}


def cpu_baseline(w, synth, oracle, qs, budget_s, threads=None):
    """The CPU oracle on bounded samples: the S smallest documents of the
    workload (their own compact plan), for S = 32 and 256, queried with the
    query set (cycled) for half the budget each.  The time per lookup is
    a + b * S (a per lookup: terms, hashing; b per document); the rate is
    extrapolated to the workload's document count along that line.  Used
    where a whole block is too large to build on the host in the run."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    if w.kind != "dna" or w.n_docs < 256:
        return None
    smallest = np.argsort(synth.doc_lengths(w), kind="stable")
    if threads is None:
        threads = min(os.cpu_count() or 1, 16)
    points, notes = [], []
    for S in (32, 256):
        texts = [synth.dna_docs(w, first=int(d), count=1).bytes.tobytes() for d in smallest[:S]]
        ix = oracle.OracleIndex(oracle.Docs.from_lists(texts), kind=oracle.DNA, q=w.q,
                                canonical=w.canonical, h=w.h, p=w.p, B=min(w.B, S) if w.B else 0,
                                seed=w.hash_seed)
        done_l, i, nq = 0, 0, qs.n
        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            while time.perf_counter() - t0 < budget_s / 2:
                batch = [qs.get(j % nq) for j in range(i, i + 4 * threads)]
                for sc, l in ex.map(ix.query_scores, batch):
                    done_l += l
                i += len(batch)
        dt = time.perf_counter() - t0
        points.append((S, dt / done_l))
        notes.append(f"{S} docs: {i} queries, {done_l / dt:.3g} lookups/s")
        del ix
    (s0, t0_), (s1, t1_) = points
    b = max((t1_ - t0_) / (s1 - s0), 0.0)
    a = max(t0_ - b * s0, 0.0)
    rate = 1.0 / (a + b * w.n_docs)
    return {"value": rate, "unit": "lookups/s", "cores": threads, "kind": "oracle",
            "sample": f"the 32 and 256 smallest documents (their own compact plan), the query "
                      f"set cycled, {budget_s / 2:.0f}s each ({'; '.join(notes)}); time per "
                      f"lookup {a * 1e9:.0f} ns + {b * 1e9:.2f} ns per document, extrapolated "
                      f"to {w.n_docs} documents"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   "multi-GPU runs are not part of this build"}))
        print("bench.py measures one GPU only (--gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1905_09624_amd as cobs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    cobs.lib()   # fails loudly when the HIP library is missing

    w = synth.CONFIGS[args.config]
    if args.scale > 1:
        w = w.scaled(args.scale)
    if args.queries:
        from dataclasses import replace
        w = replace(w, n_queries=args.queries)
    log(f"workload {w.name}: {w.n_docs} docs, B={w.B}, {w.n_queries} queries")

    t0 = time.time()
    if w.kind == "dna":
        ix = build_index_dna(cobs, synth, torch, w, int(args.chunk_gb * 2**30))
        qs = synth.dna_queries(w)
    else:
        d = synth.docs(w)
        prm = cobs.make_params(cobs.BYTES, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
        ix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
        qs = synth.text_queries(w, d)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    info = ix.info()
    blocks = [ix.block(b) for b in range(info["n_blocks"])]
    row_bytes_per_term = sum(b["stride"] for b in blocks)
    log(f"index built in {build_s:.1f}s: {info['n_blocks']} blocks, "
        f"{info['total_bytes'] / 1e9:.2f} GB, {row_bytes_per_term} row bytes per term-hash")

    if args.calib_copy_gb > 0:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE
        # counters calibrate the counter units of a --pmc run
        nb = int(args.calib_copy_gb * 2**30)
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {nb} bytes done")
        del src, dst

    # autotune the gather launch shape on a separate query set of the same shape
    if args.tuning:
        shape = [int(x) for x in args.tuning.split(",")] + [0]
        ix.set_tuning(shape[0], shape[1], shape[2])
        tuning = {"unroll": shape[0], "chunk": shape[1], "order": shape[2], "gather_ms": None}
    else:
        if w.kind == "dna":
            tq = synth.dna_queries(w, n=qs.n, first=qs.n)
        else:
            tq = synth.text_queries(w, d, n=qs.n)
        tuning = ix.tune(torch.from_numpy(tq.bytes.copy()).to("cuda"), tq.q_off)
    log(f"tuning: {tuning}")

    qdev = torch.from_numpy(qs.bytes.copy()).to("cuda")     # resident in HBM
    q_off = qs.q_off
    k = w.k

    for i in range(max(args.warmup, 1)):
        nt, hoff, ids, sc = ix.query_flat(qdev, q_off, k=k, topk=0)
        log(f"warmup {i + 1}/{args.warmup}")
    lookups = int(nt.sum())
    survivors = int(len(ids))

    cobs.profile(True)
    cobs.profile_read(reset=True)
    torch.cuda.synchronize()
    step_s = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        ix.query_flat(qdev, q_off, k=k, topk=0)   # returns after its results are on the host
        step_s.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = cobs.profile_read(reset=True)
    cobs.profile(False)
    log(f"timed {args.steps} steps in {dt:.3f}s")

    # the same step with the query bytes handed over in host memory (PCIe included)
    qhost = qs.bytes
    ix.query_flat(qhost, q_off, k=k, topk=0)
    t1 = time.perf_counter()
    for _ in range(2):
        ix.query_flat(qhost, q_off, k=k, topk=0)
    host_step_ms = (time.perf_counter() - t1) / 2 * 1e3

    ms_per_step = dt / args.steps * 1e3
    value = lookups * args.steps / dt
    gather_ms = prof["total_ms"] / max(prof["launches"], 1)
    gather_bytes = prof["row_bytes"] / max(prof["launches"], 1)
    achieved = gather_bytes / (gather_ms * 1e-3) / 1e9

    # the device's read ceiling beside it: a plain coalesced read of 8 GiB
    rbuf = torch.empty(8 << 30, dtype=torch.uint8, device="cuda")
    cobs.read_bandwidth(rbuf)
    stream_read = max(cobs.read_bandwidth(rbuf) for _ in range(3))
    # random 1 KiB row reads (the gather's access pattern, cached loads) over
    # working sets that fit each XCD's L2, the last-level cache, or only HBM
    rows_read = {label: cobs.read_rows_bandwidth(rbuf[:nb], 24 << 20, cached=True)
                 for label, nb in (("4MiB", 4 << 20), ("128MiB", 128 << 20), ("8GiB", 8 << 30))}
    del rbuf
    log(f"read ceiling {stream_read:.0f} GB/s; random rows {rows_read}")

    # top-k run of the same set (K = 0, top-100)
    topk_ms = None
    if w.topk:
        ix.query_flat(qdev, q_off, k=(0, 1), topk=w.topk)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(2):
            ix.query_flat(qdev, q_off, k=(0, 1), topk=w.topk)
        torch.cuda.synchronize()
        topk_ms = (time.perf_counter() - t1) / 2 * 1e3

    # early exit (cobs_prune): the same threshold step with pruning on, whose
    # hits must equal the unpruned step's; lookups counted the same way
    ix.set_tuning(tuning["unroll"], tuning["chunk"], tuning["order"], prune=cobs.PRUNE_ON)
    _, _, pids, pscores = ix.query_flat(qdev, q_off, k=k, topk=0)
    cobs.profile(True)
    cobs.profile_read(reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    psteps = max(args.steps // 2, 2)
    for _ in range(psteps):
        ix.query_flat(qdev, q_off, k=k, topk=0)
    torch.cuda.synchronize()
    pdt = (time.perf_counter() - t1) / psteps
    pprof = cobs.profile_read(reset=True)
    cobs.profile(False)
    ix.set_tuning(tuning["unroll"], tuning["chunk"], tuning["order"])
    pruned = {"ms_per_step": pdt * 1e3, "lookups_per_s": lookups / pdt,
              "gather_kernel_ms": pprof["total_ms"] / max(pprof["launches"], 1),
              "speedup_vs_full_scoring": ms_per_step / (pdt * 1e3),
              "same_hits": bool(np.array_equal(pids, ids) and np.array_equal(pscores, sc)),
              "steps": psteps}
    log(f"pruned step: {pruned}")

    # plain path: one query per launch, same queries
    npq = min(args.plain_queries, qs.n)
    sub = qs.subset(range(npq))
    subdev = torch.from_numpy(sub.bytes.copy()).to("cuda")
    ix.query_flat(subdev, sub.q_off, k=k, topk=0, mode=cobs.MODE_PLAIN)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pnt = ix.query_flat(subdev, sub.q_off, k=k, topk=0, mode=cobs.MODE_PLAIN)[0]
    torch.cuda.synchronize()
    plain_dt = time.perf_counter() - t1
    plain_rate = int(pnt.sum()) / plain_dt
    log(f"plain path: {npq} queries in {plain_dt:.3f}s")

    def set_launch(launch):
        ix.set_tuning(tuning["unroll"], tuning["chunk"], tuning["order"], launch=launch)

    # the plain path with every kernel launched on the stream (no replayed
    # graphs), and 1 kbp queries alone (the launch-bound case) both ways
    set_launch(cobs.LAUNCH_DIRECT)
    ix.query_flat(subdev, sub.q_off, k=k, topk=0, mode=cobs.MODE_PLAIN)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dnt = ix.query_flat(subdev, sub.q_off, k=k, topk=0, mode=cobs.MODE_PLAIN)[0]
    torch.cuda.synchronize()
    plain_direct_rate = int(dnt.sum()) / (time.perf_counter() - t1)
    one_kbp = {}
    ones = [qs.get(i)[:1000] for i in range(qs.n) if int(qs.q_off[i + 1] - qs.q_off[i]) >= 1000][:200]
    for label, launch in (("graph", cobs.LAUNCH_AUTO), ("direct", cobs.LAUNCH_DIRECT)):
        set_launch(launch)
        lat = []
        for rep in range(2):
            lat = []
            for x in ones:
                a = np.frombuffer(x, np.uint8)
                off = np.array([0, len(x)], np.uint64)
                t1 = time.perf_counter()
                ix.query_flat(a, off, k=k, mode=cobs.MODE_PLAIN)
                lat.append(time.perf_counter() - t1)
        lat = np.array(lat) * 1e3
        one_kbp[label] = {"p50_ms": float(np.percentile(lat, 50)),
                          "p99_ms": float(np.percentile(lat, 99)), "queries": len(ones)}
    set_launch(cobs.LAUNCH_AUTO)
    log(f"plain path direct launches: {plain_direct_rate:.4g} lookups/s; 1 kbp alone: {one_kbp}")

    serving = None
    if args.serve_rates and args.config == 3:
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        def set_prune(on):
            ix.set_tuning(tuning["unroll"], tuning["chunk"], tuning["order"],
                          prune=cobs.PRUNE_ON if on else cobs.PRUNE_OFF)

        serving = serve_measure(cobs, synth, torch, ix, rates, args.serve_pool,
                                args.serve_seconds, args.serve_max, 100, args.serve_streams,
                                set_launch, set_prune)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = min(os.cpu_count() or 1, 16)
        if w.kind == "dna" and w.B == 8192 and args.scale == 1:
            order, n_terms = ix.order()
            cpu = cpu_baseline_block(w, synth, oracle, qs, order, n_terms, args.cpu_seconds, threads)
            log(f"cpu baseline ({threads} threads): {cpu['sample']}")
        else:
            cpu = cpu_baseline(w, synth, oracle, qs, args.cpu_seconds, threads)
            one = cpu_baseline(w, synth, oracle, qs, args.cpu_seconds / 2, threads=1)
            if cpu and one:
                cpu["value_1_thread"] = one["value"]
                cpu["sample_1_thread"] = one["sample"]
        try:
            import psutil
            cpu["host_ram_gb"] = psutil.virtual_memory().total / 1e9
        except Exception:
            pass
        log("cpu baseline done")

    offload = None
    if args.offload_gb > 0 and 2 * max(b["rows"] * b["stride"] for b in blocks) <= args.offload_gb * 1e9:
        # out of core: the matrix in pinned host memory, streamed per batch
        t1 = time.time()
        try:
            ix.offload(int(args.offload_gb * 1e9))
        except cobs.CobsError as e:
            offload = {"error": str(e)}
    if offload is None and ix.info()["host_resident"]:
        oinfo = ix.info()
        log(f"offloaded in {time.time() - t1:.1f}s: {oinfo['n_groups']} groups, "
            f"staging 2 x {oinfo['stage_bytes'] / 1e9:.2f} GB")
        _, _, oids, oscores = ix.query_flat(qdev, q_off, k=k)
        same = bool(np.array_equal(oids, ids) and np.array_equal(oscores, sc))
        cobs.profile(True)
        cobs.profile_read(reset=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(2):
            ix.query_flat(qdev, q_off, k=k)
        torch.cuda.synchronize()
        odt = (time.perf_counter() - t1) / 2
        oprof = cobs.profile_read(reset=True)
        cobs.profile(False)
        ogather = oprof["total_ms"] / max(oprof["launches"], 1)
        offload = {"device_budget_gb": args.offload_gb, "groups": oinfo["n_groups"],
                   "stage_bytes": oinfo["stage_bytes"], "ms_per_step": odt * 1e3,
                   "lookups_per_s": lookups / odt, "gather_ms": ogather, "same_hits": same,
                   "host_link_GBps": info["total_bytes"] / (ogather * 1e-3) / 1e9,
                   "mode": "streamed (automatic choice for this batch)"}
        # small batches read their rows in place from host memory (automatic
        # below the matrix's bytes); the same queries against the in-HBM hits
        small = []
        for nq in (1, 10, 100, 1000):
            sq = qs.subset(range(min(nq, qs.n)))
            sdev = torch.from_numpy(sq.bytes.copy()).to("cuda")
            ix.set_tuning(0, 0, 0, cobs.HOST_READS_AUTO)
            got = ix.query_flat(sdev, sq.q_off, k=k)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(3):
                ix.query_flat(sdev, sq.q_off, k=k)
            torch.cuda.synchronize()
            sdt = (time.perf_counter() - t1) / 3
            ix.set_tuning(0, 0, 0, cobs.HOST_READS_STREAM)
            t1 = time.perf_counter()
            st_res = ix.query_flat(sdev, sq.q_off, k=k)
            torch.cuda.synchronize()
            stream_dt = time.perf_counter() - t1
            ix.set_tuning(0, 0, 0, cobs.HOST_READS_AUTO)
            nt_s = int(got[0].sum())
            small.append({"queries": sq.n, "distinct_terms": nt_s, "ms_per_batch": sdt * 1e3,
                          "streamed_ms_per_batch": stream_dt * 1e3,
                          "rows_GBps": nt_s * w.h * row_bytes_per_term / sdt / 1e9,
                          "same_hits_as_streamed": bool(all(np.array_equal(a, b)
                                                            for a, b in zip(got, st_res)))})
            log(f"offloaded, in place: {small[-1]}")
        offload["in_place"] = small
        log(f"offloaded: {offload}")

    traffic = committed_traffic(w.name)
    out = {
        "metric": "k-mer lookups/s (distinct query terms scored against every document) "
                  "+ row-gather HBM GB/s",
        "value": value,
        "unit": "lookups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "median_ms_per_step": float(np.median(step_s) * 1e3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": w.name + (" (paper's 100k-document compact shape, synthetic random "
                                  "ACGT)" if args.config == 3 and args.scale == 1 else ""),
            "documents": w.n_docs, "block_docs": w.B, "q": w.q, "h": w.h, "fpr": w.p,
            "queries": qs.n, "distinct_terms": lookups, "threshold": f"{k[0]}/{k[1]}",
            "index_bytes": info["total_bytes"], "blocks": info["n_blocks"],
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
        },
        "hbm": {
            "stream_read_GBps": stream_read,
            "random_rows_GBps": rows_read,
            "gather_frac_of_stream_read": achieved / stream_read,
            "gather_counted_GBps": traffic / (gather_ms * 1e-3) / 1e9 if traffic else None,
        },
        "row_fetches_per_s": value * w.h * info["n_blocks"],
        "gather_kernel_ms": gather_ms,
        "host_input_ms_per_step": host_step_ms,
        "tuning": tuning,
        "gather_row_bytes_per_launch": gather_bytes,
        "survivors_per_step": survivors,
        "topk100_ms_per_step": topk_ms,
        "pruned": pruned,
        "plain_path": {"value": plain_rate, "unit": "lookups/s", "queries": npq,
                       "speedup_batched": value / plain_rate if plain_rate else None,
                       "direct_launches_value": plain_direct_rate,
                       "one_kbp_latency": one_kbp},
        "build_s": build_s,
        "serving": serving,
        "out_of_core": offload,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
