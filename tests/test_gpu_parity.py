"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element, on seeded inputs.  Integer results: bit-exact."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _cobs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_09624_amd as cobs
    return cobs


def build_both(docs, kind, q, canonical, h, p, B, seed):
    cobs = _cobs()
    prm = cobs.make_params(kind, q, canonical, h, p, B, seed)
    gix = cobs.Index.build(prm, docs.bytes, docs.str_off, docs.doc_str)
    oix = oracle.OracleIndex(oracle.Docs(docs.bytes, docs.str_off, docs.doc_str), kind=kind, q=q,
                             canonical=canonical, h=h, p=p, B=B, seed=seed)
    return gix, oix


def assert_same_index(gix, oix):
    order, nterms = gix.order()
    assert np.array_equal(nterms, oix.n_terms())
    assert np.array_equal(order, oix.order())
    assert gix.info()["n_blocks"] == oix.n_blocks
    omat = oix.matrix()
    for b in range(oix.n_blocks):
        gb, ob = gix.block(b), oix.block(b)
        for k in ("first", "docs", "rows", "stride"):
            assert gb[k] == ob[k], (b, k)
        n = ob["rows"] * ob["stride"]
        assert np.array_equal(gix.read(gb["offset"], n), omat[ob["offset"]:ob["offset"] + n]), b


def queries_of(strings):
    data = b"".join(strings)
    off = np.zeros(len(strings) + 1, np.uint64)
    off[1:] = np.cumsum([len(s) for s in strings])
    return np.frombuffer(data, np.uint8).copy() if data else np.zeros(0, np.uint8), off


def rand_dna(rng, n, alphabet=b"ACGT"):
    return bytes(rng.choice(np.frombuffer(alphabet, np.uint8), size=n))


def check_queries(gix, oix, data, off, k=(4, 5), topk=0, mode=0, chunk=0):
    res = gix.query(data, off, k=k, topk=topk, mode=mode, chunk=chunk)
    for i in range(len(off) - 1):
        qb = data[int(off[i]):int(off[i + 1])].tobytes()
        ids, sc, l = oix.query(qb, k[0], k[1], topk)
        gids, gsc, gl = res[i]
        assert gl == l, (i, gl, l)
        assert np.array_equal(gids, ids), (i, gids[:10], ids[:10])
        assert np.array_equal(gsc, sc), i


# ---- construction -----------------------------------------------------------

@pytest.mark.parametrize("case", [
    dict(kind=0, q=31, canonical=True, h=1, p=0.3, B=0),
    dict(kind=0, q=31, canonical=True, h=1, p=0.3, B=8),
    dict(kind=0, q=11, canonical=False, h=3, p=0.1, B=5),
    dict(kind=1, q=8, canonical=False, h=3, p=0.1, B=16),
    dict(kind=1, q=3, canonical=False, h=2, p=0.3, B=0),
])
def test_build_matrix_bitexact(case):
    rng = np.random.default_rng(5)
    docs = []
    for i in range(37):
        n = int(rng.integers(0, 3000))
        if case["kind"] == 0:
            alph = b"ACGTN" if i % 5 == 0 else b"acgtACGT"
            docs.append([rand_dna(rng, n, alph), rand_dna(rng, n // 3)])
        else:
            docs.append([bytes(rng.integers(0, 256, n, dtype=np.uint8))])
    d = oracle.Docs.from_lists(docs)
    gix, oix = build_both(d, seed=99, **case)
    assert_same_index(gix, oix)


def test_build_wide_classic_block_multiple_slices():
    # 9000 documents in one classic block: 1128-byte rows, two column slices
    rng = np.random.default_rng(8)
    d = oracle.Docs.from_lists([rand_dna(rng, int(rng.integers(31, 80))) for _ in range(9000)])
    gix, oix = build_both(d, 0, 31, True, 1, 0.3, 0, 7)
    assert_same_index(gix, oix)
    data, off = queries_of([rand_dna(rng, 200) for _ in range(5)] +
                           [d.bytes[int(d.str_off[j]):int(d.str_off[j + 1])].tobytes()
                            for j in (0, 4000, 8999)])
    sc, l = gix.scores(data, off)
    for i in range(len(off) - 1):
        want, wl = oix.query_scores(data[int(off[i]):int(off[i + 1])].tobytes())
        assert wl == l[i]
        assert np.array_equal(sc[i], want)
    check_queries(gix, oix, data, off, k=(1, 2))


def test_streamed_build_equals_one_call():
    cobs = _cobs()
    w = synth.CONFIGS[3].scaled(500)
    d = synth.docs(w)
    prm = cobs.make_params(0, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    one = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    n = d.n_docs
    cuts = [0, 17, 18, 90, n]

    def runs(pass_no):
        order = range(len(cuts) - 1) if pass_no == 0 else reversed(range(len(cuts) - 1))
        for k in order:
            a, b = cuts[k], cuts[k + 1]
            sub = synth.dna_docs(w, first=a, count=b - a)
            yield a, sub.bytes, sub.str_off, sub.doc_str

    two = cobs.Index.build_streamed(prm, n, runs)
    assert one.info() == two.info()
    nb = one.info()["total_bytes"]
    assert np.array_equal(one.read(0, nb), two.read(0, nb))


# ---- query steps -----------------------------------------------------------------

def test_terms_and_dedup_match_oracle():
    cobs = _cobs()
    rng = np.random.default_rng(2)
    d = oracle.Docs.from_lists([rand_dna(rng, 500)])
    prm = cobs.make_params(0, 31, True, 1, 0.3, 0, 1)
    gix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    # the last three: longer than an LDS set (their windows partitioned by
    # hash into LDS sets), one with a k-mer repeated past an LDS table's
    # capacity in one partition (the device table instead)
    qs = [b"", b"ACGT", rand_dna(rng, 31), rand_dna(rng, 5000, b"ACGTN"),
          rand_dna(rng, 200) * 5, b"acgtNNACGTAC" * 40, rand_dna(rng, 20000),
          rand_dna(rng, 70000, b"ACGTN"), rand_dna(rng, 3000) + b"A" * 20000 + rand_dna(rng, 3000)]
    data, off = queries_of(qs)
    got = gix.terms(data, off, q=31)
    for i, s in enumerate(qs):
        want = oracle.unique(oracle.terms(0, 31, True, s))
        assert np.array_equal(np.sort(got[i]), want), i


def test_bytes_terms_with_all_ones_term():
    cobs = _cobs()
    d = oracle.Docs.from_lists([b"\xff" * 40 + b"abcdefghij"])
    prm = cobs.make_params(1, 8, False, 3, 0.1, 0, 3)
    gix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    rng = np.random.default_rng(12)
    # the last query: a global dedup table spread over several workgroups,
    # with the all-ones term in more than one of them
    long_q = (b"\xff" * 9000 + rng.integers(0, 256, 12000, dtype=np.uint8).tobytes()
              + b"\xff" * 9000)
    # and a query partitioned into LDS sets with the all-ones term in one
    mid_q = (rng.integers(0, 256, 15000, dtype=np.uint8).tobytes() + b"\xff" * 40
             + rng.integers(0, 256, 15000, dtype=np.uint8).tobytes())
    qs = [b"\xff" * 20, b"\xff" * 9 + b"abc", b"xyz", long_q, mid_q]
    data, off = queries_of(qs)
    got = gix.terms(data, off, q=8)
    for i, s in enumerate(qs):
        assert np.array_equal(np.sort(got[i]), oracle.unique(oracle.terms(1, 8, False, s)))
    assert gix.order()[1][0] == 3 + 8   # distinct 8-grams of the document


@pytest.mark.parametrize("kind", ["dna", "bytes"])
def test_terms_of_a_batch_of_millions_of_windows(kind):
    # over 8.4 million windows in one batch: each lane of the extract kernel
    # takes 16 consecutive windows, and many lanes hold the end of one query
    # and the start of the next (queries of 0 to 40 bytes among long ones)
    cobs = _cobs()
    rng = np.random.default_rng(21)
    if kind == "dna":
        q, prm, doc = 31, cobs.make_params(0, 31, True, 1, 0.3, 0, 1), rand_dna(rng, 500)
        alphabet = np.frombuffer(b"ACGTacgt" * 8 + b"N", np.uint8)
        gen = lambda n: rng.choice(alphabet, n).tobytes()
    else:
        q, prm, doc = 8, cobs.make_params(1, 8, False, 3, 0.1, 0, 3), b"abcdefghijklmnop"
        gen = lambda n: rng.integers(0, 256, n, dtype=np.uint8).tobytes()
    d = oracle.Docs.from_lists([doc])
    gix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    qs, windows = [], 0
    while windows < 9_000_000:
        r = rng.random()
        n = int(rng.integers(0, 41) if r < 0.4 else rng.integers(41, 300) if r < 0.7
                else rng.integers(300, 60000))
        qs.append(gen(n))
        windows += max(n - q + 1, 0)
    data, off = queries_of(qs)
    got = gix.terms(data, off, q=q)
    for i, s in enumerate(qs):
        want = oracle.unique(oracle.terms(0 if kind == "dna" else 1, q, kind == "dna", s))
        assert np.array_equal(np.sort(got[i]), want), (i, len(s))


def test_index_from_fasta_files_with_many_reads(tmp_path):
    # documents read from FASTA files: every read is a string of its document
    # (no k-mer spans two reads); the index and hits equal the oracle's over
    # the same strings, and multi-FASTA query files give one query per record
    cobs = _cobs()
    rng = np.random.default_rng(13)
    ds = cobs.DocSet()
    for d in range(9):
        reads = [rand_dna(rng, int(rng.integers(20, 400)), b"ACGTacgtN") for _ in range(int(rng.integers(1, 30)))]
        path = tmp_path / f"doc{d}.fa"
        path.write_bytes(b"".join(b">r%d\n%s\n" % (i, r) for i, r in enumerate(reads)))
        ds.add_file(str(path), cobs.FASTA)
    data, so, dstr = ds.arrays()
    docs = oracle.Docs(data, so, dstr)
    gix, oix = build_both(docs, 0, 15, True, 2, 0.2, 4, 5)
    assert_same_index(gix, oix)
    picks = [data[int(so[s]):int(so[s + 1])].tobytes() for s in (0, 3, 7, 20)]
    qfile = tmp_path / "queries.fa"
    qfile.write_bytes(b"".join(b">q%d\n%s\n" % (i, q) for i, q in enumerate(picks)))
    qd, qso, qds = cobs.DocSet().add_file(str(qfile), cobs.MULTI_FASTA).arrays()
    assert len(qds) == len(picks) + 1
    check_queries(gix, oix, qd, qso, k=(1, 2), topk=0)
    check_queries(gix, oix, qd, qso, k=(0, 1), topk=3, mode=1)


# ---- scores and hits on scaled workloads -------------------------------------------

WORKLOADS = {
    "classic-1k/s4": (synth.CONFIGS[1].scaled(4), 40),
    "classic-10k/s20": (synth.CONFIGS[2].scaled(20), 40),
    "compact-100k/s100": (synth.CONFIGS[3].scaled(100), 40),
    "text-50k/s50": (synth.CONFIGS[4].scaled(50), 60),
}


@pytest.fixture(scope="module", params=sorted(WORKLOADS))
def workload(request):
    w, nq = WORKLOADS[request.param]
    d = synth.docs(w)
    qs = synth.dna_queries(w, n=nq) if w.kind == "dna" else synth.text_queries(w, d, n=nq)
    kind = 0 if w.kind == "dna" else 1
    gix, oix = build_both(d, kind, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    return w, d, qs, gix, oix


def test_workload_index_bitexact(workload):
    w, d, qs, gix, oix = workload
    assert_same_index(gix, oix)


def test_workload_full_scores(workload):
    w, d, qs, gix, oix = workload
    sc, l = gix.scores(qs.bytes, qs.q_off)
    for i in range(qs.n):
        want, wl = oix.query_scores(qs.get(i))
        assert l[i] == wl
        assert np.array_equal(sc[i], want), i


@pytest.mark.parametrize("k,topk", [((4, 5), 0), ((0, 1), 10), ((1, 2), 3), ((0, 1), 0)])
@pytest.mark.parametrize("mode", [0, 1])
def test_workload_hits(workload, k, topk, mode):
    w, d, qs, gix, oix = workload
    check_queries(gix, oix, qs.bytes, qs.q_off, k=k, topk=topk, mode=mode)


# ---- early exit of threshold queries (cobs_prune) ----------------------------------
# Pruning runs in unpacked launches only: an index with a block wider than
# 4,096 documents (1 KiB row slices).

@pytest.fixture(scope="module", params=["dna-h1", "bytes-h3"])
def wide(request):
    # 9,000 short documents in blocks of 8,192 (one 1 KiB slice and a narrow
    # last block); queries: exact substrings of documents, substrings with 1%
    # substitutions, random strings, and the empty query
    cobs = _cobs()
    rng = np.random.default_rng(31)
    dna = request.param == "dna-h1"
    gen = (lambda n: rand_dna(rng, n)) if dna else (lambda n: rng.integers(0, 256, n, np.uint8).tobytes())
    docs = [[gen(int(rng.integers(40, 600)))] for _ in range(9000)]
    kind, q, h, p = (0, 31, 1, 0.3) if dna else (1, 8, 3, 0.1)
    gix, oix = build_both(oracle.Docs.from_lists(docs), kind, q, dna, h, p, 8192, 0xABC)
    assert max(gix.block(b)["stride"] for b in range(gix.info()["n_blocks"])) == 1024
    qs, src = [b""], [-1]
    for i in range(60):
        if i % 3 == 2:
            qs.append(gen(int(rng.integers(q, 600))))
            src.append(-1)
            continue
        j = int(rng.integers(0, len(docs)))
        x = bytearray(docs[j][0])
        L = int(rng.integers(min(len(x), 95), len(x) + 1))
        a = int(rng.integers(0, len(x) - L + 1))
        x = x[a:a + L]
        if i % 3 == 1:
            for t in np.nonzero(rng.random(len(x)) < 0.01)[0]:
                x[t] = (b"ACGT"[(b"ACGT".index(x[t]) + 1) % 4]) if dna else (x[t] + 1) % 256
        qs.append(bytes(x))
        src.append(j if i % 3 == 0 else -1)
    data, off = queries_of(qs)
    return cobs, gix, oix, data, off, src


@pytest.mark.parametrize("k,topk,chunk", [((4, 5), 0, 0), ((1, 2), 3, 0), ((4, 5), 0, 37),
                                           ((1, 2), 0, 37), ((9, 10), 5, 100), ((1, 1), 0, 0),
                                           ((1, 1), 0, 64), ((0, 1), 10, 0)])
@pytest.mark.parametrize("mode", [0, 1])
def test_pruned_hits_equal_oracle(wide, k, topk, chunk, mode):
    # the same hits, scores and top-k as the oracle with pruning on, whole
    # queries and queries split into chunks of 37, 64 or 100 terms (their
    # counts merged through the score buffer; split queries run in two
    # launches, and at K = 1/2 the shorter ones whole in the first).  K = 1:
    # T = l, so after c terms
    # a document stays live only with a score of exactly c, and a document
    # holding the whole query must still be found (an off-by-one in the bound
    # would drop it)
    cobs, gix, oix, data, off, src = wide
    gix.set_tuning(prune=cobs.PRUNE_ON)
    try:
        check_queries(gix, oix, data, off, k=k, topk=topk, mode=mode, chunk=chunk)
        if k == (1, 1):
            got = gix.query(data, off, k=k, mode=mode, chunk=chunk)
            for i, j in enumerate(src):
                if j >= 0:
                    assert j in set(got[i][0].tolist()), (i, j)
    finally:
        gix.set_tuning()


def test_pruned_results_equal_unpruned(wide):
    # pruning never changes a result, and full score vectors ignore it
    cobs, gix, oix, data, off, src = wide
    want = [gix.query(data, off, k=k, topk=t) for k, t in (((4, 5), 0), ((1, 2), 2))]
    sc0 = gix.scores(data, off)
    gix.set_tuning(prune=cobs.PRUNE_ON)
    try:
        got = [gix.query(data, off, k=k, topk=t) for k, t in (((4, 5), 0), ((1, 2), 2))]
        sc1 = gix.scores(data, off)
    finally:
        gix.set_tuning()
    for x, y in zip(want, got):
        for u, v in zip(x, y):
            assert np.array_equal(u[0], v[0]) and np.array_equal(u[1], v[1]) and u[2] == v[2]
    assert np.array_equal(sc0[0], sc1[0]) and np.array_equal(sc0[1], sc1[1])
    with pytest.raises(cobs.CobsError) as e:
        gix.set_tuning(prune=2)
    assert e.value.status == cobs.EINVAL


def test_planted_source_never_missed(workload):
    # no false negatives: the source document scores at least the exact overlap
    w, d, qs, gix, oix = workload
    sc, l = gix.scores(qs.bytes, qs.q_off)
    kind = 0 if w.kind == "dna" else 1
    all_docs = oracle.Docs(d.bytes, d.str_off, d.doc_str)
    for i in range(qs.n):
        if qs.src[i] < 0:
            continue
        s = int(qs.src[i])
        ex, _ = oracle.exact_intersection(all_docs, qs.get(i), kind=kind, q=w.q,
                                          canonical=w.canonical)
        assert sc[i][s] >= ex[s]
        assert np.all(sc[i] >= ex)


def test_single_queries_replayed_graphs_equal_direct_and_oracle(workload):
    # single short queries run as replayed hipGraphs (one per launch-shape
    # class); every replay is checked against the oracle and the direct
    # launches, with batched work and synchronisations between the replays,
    # each class replayed many times, and one query too long for a graph
    import torch
    cobs = _cobs()
    w, d, qs, gix, oix = workload
    rng = np.random.default_rng(11)
    base = [qs.get(i) for i in range(qs.n)]
    strings = [b""]
    for L in (31, 40, 100, 200, 500, 1000, 2500, 4000, 6000, 8200, 9000):
        s = base[int(rng.integers(0, len(base)))]
        strings.append((s * (L // max(len(s), 1) + 1))[:L])
    strings += base[:8]
    want = {}
    # the last two with early exit: split queries gather twice in the graph
    for k, topk, prune in (((4, 5), 0, 0), ((0, 1), 5, 0), ((4, 5), 0, 1), ((9, 10), 3, 1)):
        for rep in range(3):
            for x in strings:
                data = np.frombuffer(x, np.uint8) if x else np.zeros(0, np.uint8)
                off = np.array([0, len(x)], np.uint64)
                got = {}
                for launch in (cobs.LAUNCH_AUTO, cobs.LAUNCH_DIRECT):
                    gix.set_tuning(launch=launch, prune=prune)
                    got[launch] = gix.query(data, off, k=k, topk=topk)[0]
                gix.set_tuning()
                kk = (x, k, topk)
                if kk not in want:
                    want[kk] = oix.query(x, k[0], k[1], topk)
                ids, sc, l = want[kk]
                for g in got.values():
                    assert g[2] == l and np.array_equal(g[0], ids) and np.array_equal(g[1], sc), (len(x), k)
            # eager batched work between the rounds of replays
            gix.query(qs.bytes, qs.q_off, k=(1, 2))
            torch.cuda.synchronize()


# ---- edge cases -----------------------------------------------------------------

def test_edge_queries():
    rng = np.random.default_rng(4)
    docs = oracle.Docs.from_lists([rand_dna(rng, int(rng.integers(100, 4000))) for _ in range(25)]
                                  + [b"", b"ACG", b"N" * 100])
    gix, oix = build_both(docs, 0, 31, True, 1, 0.3, 6, 11)
    assert_same_index(gix, oix)
    src = docs.bytes[int(docs.str_off[3]):int(docs.str_off[4])].tobytes()
    qs = [b"", b"A" * 30, b"N" * 64, src, src[:31], src * 3, rand_dna(rng, 9000),
          src[:500] + b"N" + src[500:], b"ACGT" * 2000]
    data, off = queries_of(qs)
    for k, topk in (((4, 5), 0), ((0, 1), 5), ((1, 1), 0), ((3, 2), 0)):
        check_queries(gix, oix, data, off, k=k, topk=topk, mode=0)
        check_queries(gix, oix, data, off, k=k, topk=topk, mode=1)
    assert gix.query(data[:0], np.zeros(1, np.uint64)) == []


def test_long_query_multi_chunk_and_global_table():
    # > 12,288 windows: dedup table in global memory (> 16384: several
    # workgroups); 4,097-12,288 windows: the 128 KiB LDS table (12,000: load
    # 0.73); > 1024 terms: several chunks merged by the last wavefront of
    # each (query, slice)
    rng = np.random.default_rng(6)
    docs = oracle.Docs.from_lists([rand_dna(rng, 30000) for _ in range(12)])
    gix, oix = build_both(docs, 0, 31, True, 1, 0.3, 4, 2)
    d0 = docs.bytes[int(docs.str_off[0]):int(docs.str_off[1])].tobytes()
    qs = [d0[:20000] + rand_dna(rng, 30000), rand_dna(rng, 70000), d0, d0[:6000],
          rand_dna(rng, 12000), rand_dna(rng, 14000)]
    data, off = queries_of(qs)
    sc, l = gix.scores(data, off)
    for i, s in enumerate(qs):
        want, wl = oix.query_scores(s)
        assert l[i] == wl
        assert np.array_equal(sc[i], want)
    check_queries(gix, oix, data, off, k=(1, 5), topk=0, mode=0)
    check_queries(gix, oix, data, off, k=(0, 1), topk=7, mode=1)
    # each query in a single work item (no merge) and in many small ones
    for chunk in (1 << 20, 300):
        res = gix.query(data, off, k=(1, 5), chunk=chunk)
        for i, s in enumerate(qs):
            ids, sc, l = oix.query(s, 1, 5, 0)
            assert res[i][2] == l and np.array_equal(res[i][0], ids) and np.array_equal(res[i][1], sc)


def test_very_long_queries_use_wide_counters():
    # 1.1 M and 16.8 M distinct terms: 24 and 32 counter planes, dedup over
    # many workgroups, thousands of chunks per (query, slice)
    rng = np.random.default_rng(31)
    docs = oracle.Docs.from_lists([rand_dna(rng, int(n)) for n in rng.integers(20000, 60000, 10)])
    gix, oix = build_both(docs, 0, 31, True, 1, 0.3, 4, 9)
    d0 = docs.bytes[int(docs.str_off[0]):int(docs.str_off[1])].tobytes()
    qs = [d0 + rand_dna(rng, 1_100_000), rand_dna(rng, (1 << 24) + 200_000)]
    data, off = queries_of(qs)
    sc, l = gix.scores(data, off)
    hits = gix.query(data, off, k=(1, 100), topk=3)
    for i, q in enumerate(qs):
        want, wl = oix.query_scores(q)
        assert l[i] == wl and np.array_equal(sc[i], want), i
        ids, scores = oracle.report(want, wl, 1, 100, 3)
        assert np.array_equal(hits[i][0], ids) and np.array_equal(hits[i][1], scores), i


@pytest.mark.parametrize("unroll,chunk,order", [(4, 32, 1), (8, 100, 2), (4, 1024, 1), (8, 7, 1),
                                                (8, 7, 2), (8, 1 << 20, 1), (4, 1 << 20, 2)])
def test_launch_shapes_give_identical_results(workload, unroll, chunk, order):
    # every instantiated unroll, both work-item orders (query-major 1,
    # slice-major 2) and several term-chunk sizes (many merges at chunk 7,
    # every query in one work item at 2^20) give the oracle's scores (K = 0
    # reports every document with its score) and hits
    w, d, qs, gix, oix = workload
    if w.h > 1:
        unroll //= 2
    gix.set_tuning(unroll, 0, order)
    try:
        res = gix.query(qs.bytes, qs.q_off, k=(0, 1), chunk=chunk)
        for i in range(qs.n):
            want, wl = oix.query_scores(qs.get(i))
            ids, sc, l = res[i]
            assert l == wl, (unroll, chunk, order, i)
            full = np.zeros_like(want)
            full[ids] = sc
            assert len(ids) == (len(want) if wl else 0)
            if wl:
                assert np.array_equal(full, want), (unroll, chunk, order, i)
        res = gix.query(qs.bytes, qs.q_off, k=(1, 2), topk=4, chunk=chunk)
        for i in range(qs.n):
            ids, sc, l = oix.query(qs.get(i), 1, 2, 4)
            assert res[i][2] == l and np.array_equal(res[i][0], ids), (unroll, chunk, order, i)
            assert np.array_equal(res[i][1], sc), (unroll, chunk, order, i)
    finally:
        gix.set_tuning(0, 0)


def test_tuned_chunk_caps_the_split(workload):
    # a tuned chunk is the largest work item; any cap gives the same hits
    w, d, qs, gix, oix = workload
    base = gix.query(qs.bytes, qs.q_off, k=(1, 2))
    for cap in (7, 64, 1 << 20):
        gix.set_tuning(0, cap)
        try:
            got = gix.query(qs.bytes, qs.q_off, k=(1, 2))
        finally:
            gix.set_tuning(0, 0)
        for x, y in zip(base, got):
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


def test_concurrent_queries_from_threads(workload):
    # query calls on one index from several threads at once, each on its own
    # stream (each call takes its own workspace), give the single-thread hits
    import threading
    import torch
    w, d, qs, gix, oix = workload
    want = [gix.query(qs.bytes, qs.q_off, k=(1, 2)), gix.query(qs.bytes, qs.q_off, k=(0, 1), topk=3)]
    errors = []

    def worker(t):
        try:
            st = torch.cuda.Stream()
            for rep in range(4):
                j = (t + rep) % 2
                got = gix.query(qs.bytes, qs.q_off, k=((1, 2), (0, 1))[j], topk=(0, 3)[j], stream=st)
                for x, y in zip(got, want[j]):
                    if not (np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) and x[2] == y[2]):
                        errors.append((t, rep))
                        return
        except Exception as e:   # reported below
            errors.append((t, repr(e)))

    ths = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert not errors, errors


def test_set_tuning_refuses_unknown_order(workload):
    cobs = _cobs()
    w, d, qs, gix, oix = workload
    with pytest.raises(cobs.CobsError) as e:
        gix.set_tuning(0, 0, 3)
    assert e.value.status == cobs.EINVAL


def test_autotune_keeps_results(workload):
    w, d, qs, gix, oix = workload
    before = gix.query(qs.bytes, qs.q_off, k=(1, 2))
    t = gix.tune(qs.bytes, qs.q_off)
    assert t["gather_ms"] > 0 and t["unroll"] in ((4, 8) if w.h == 1 else (2, 4))
    assert t["order"] in (_cobs().ORDER_QUERIES, _cobs().ORDER_SLICES)
    after = gix.query(qs.bytes, qs.q_off, k=(1, 2))
    for x, y in zip(before, after):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    gix.set_tuning(0, 0)


def test_hits_and_flat_results_agree(workload):
    # cobs_query_batch (one cobs_hits per query) and cobs_query_results (flat)
    w, d, qs, gix, oix = workload
    for mode in (0, 1):
        a = gix.query_hits(qs.bytes, qs.q_off, k=(1, 2), topk=5, mode=mode)
        b = gix.query(qs.bytes, qs.q_off, k=(1, 2), topk=5, mode=mode)
        assert len(a) == len(b) == qs.n
        for x, y in zip(a, b):
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) and x[2] == y[2]


def test_device_resident_queries():
    import torch
    cobs = _cobs()
    w = synth.CONFIGS[3].scaled(500)
    d = synth.docs(w)
    qs = synth.dna_queries(w, n=12)
    prm = cobs.make_params(0, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    gix = cobs.Index.build(prm, d.bytes, d.str_off, d.doc_str)
    host = gix.query(qs.bytes, qs.q_off, k=(1, 2))
    dev = gix.query(torch.from_numpy(qs.bytes.copy()).cuda(), qs.q_off, k=(1, 2))
    for x, y in zip(host, dev):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) and x[2] == y[2]


def test_block_offsets_beyond_2_and_4_gib():
    # Regression: slice base offsets with bit 31 (and bit 32) set must not be
    # sign-extended.  p = 1e-5 inflates the filters: three one-document
    # blocks of ~2.6-3.1 GB, so blocks 1 and 2 start past 2^31 and 2^32 bytes.
    rng = np.random.default_rng(31)
    lists = [rand_dna(rng, 230), rand_dna(rng, 250), rand_dna(rng, 270)]
    d = oracle.Docs.from_lists(lists)
    gix, oix = build_both(d, 0, 31, True, 1, 1e-5, 1, 17)
    offs = [gix.block(b)["offset"] for b in range(3)]
    assert offs[1] >= 2**31 and offs[2] >= 2**32
    for b in range(3):
        gb, ob = gix.block(b), oix.block(b)
        assert (gb["rows"], gb["stride"], gb["docs"]) == (ob["rows"], ob["stride"], ob["docs"])
    # the rows the oracle set, read back from the device
    omat_bits = oix.matrix()
    for b in range(3):
        ob = oix.block(b)
        blk = omat_bits[ob["offset"]:ob["offset"] + ob["rows"] * ob["stride"]].reshape(ob["rows"], ob["stride"])
        rows = np.nonzero(blk[:, 0])[0]
        assert len(rows) > 150
        for r in rows[:20]:
            got = gix.read(gix.block(b)["offset"] + int(r) * ob["stride"], ob["stride"])
            assert np.array_equal(got, blk[r])
    qs = lists + [lists[1][10:200], lists[2][:100] + rand_dna(rng, 60), rand_dna(rng, 300)]
    data, off = queries_of(qs)
    sc, l = gix.scores(data, off)
    for i, s in enumerate(qs):
        want, wl = oix.query_scores(s)
        assert l[i] == wl and np.array_equal(sc[i], want), i
    check_queries(gix, oix, data, off, k=(4, 5), topk=0, mode=0)
    check_queries(gix, oix, data, off, k=(0, 1), topk=2, mode=1)


def test_score_width_overflow():
    cobs = _cobs()
    rng = np.random.default_rng(9)
    docs = oracle.Docs.from_lists([rand_dna(rng, 200)])
    prm = cobs.make_params(0, 31, True, 1, 0.3, 0, 1)
    gix = cobs.Index.build(prm, docs.bytes, docs.str_off, docs.doc_str)
    data, off = queries_of([rand_dna(rng, 70000)])
    with pytest.raises(cobs.CobsError) as e:
        gix.query(data, off, score_bits=16)
    assert e.value.status == cobs.EOVERFLOW
    gix.query(data, off, score_bits=32)


def test_invalid_arguments():
    cobs = _cobs()
    docs = oracle.Docs.from_lists([b"ACGT" * 20])
    for bad in (dict(q=32), dict(q=0), dict(h=0), dict(h=9), dict(p=0.0), dict(p=1.0)):
        kw = dict(kind=0, q=31, canonical=True, h=1, p=0.3, B=0, seed=1)
        kw.update(bad)
        with pytest.raises(cobs.CobsError) as e:
            cobs.Index.build(cobs.make_params(**kw), docs.bytes, docs.str_off, docs.doc_str)
        assert e.value.status == cobs.EINVAL
    gix = cobs.Index.build(cobs.make_params(0, 31, True, 1, 0.3, 0, 1), docs.bytes,
                           docs.str_off, docs.doc_str)
    data, off = queries_of([b"ACGT" * 10])
    with pytest.raises(cobs.CobsError):
        gix.query(data, off, k=(1, 0))
    with pytest.raises(cobs.CobsError):
        gix.query(data, off, score_bits=8)


def test_config1_full_size():
    # the classic 1,000-document workload at its full size: every query, every
    # document, threshold 0.8 with 16-bit scores
    w = synth.CONFIGS[1]
    d = synth.docs(w)
    qs = synth.dna_queries(w)
    gix, oix = build_both(d, 0, w.q, w.canonical, w.h, w.p, w.B, w.hash_seed)
    assert_same_index(gix, oix)
    sc, l = gix.scores(qs.bytes, qs.q_off)
    for i in range(qs.n):
        want, wl = oix.query_scores(qs.get(i))
        assert l[i] == wl and np.array_equal(sc[i], want), i
    res = gix.query(qs.bytes, qs.q_off, k=w.k, topk=0, score_bits=16)
    for i in range(qs.n):
        ids, s, l = oix.query(qs.get(i), w.k[0], w.k[1], 0)
        assert np.array_equal(res[i][0], ids) and np.array_equal(res[i][1], s)
