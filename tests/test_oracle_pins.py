"""Pins of the CPU oracle against facts that do not come from the oracle:
values the paper prints, closed forms, published test vectors, brute force on
tiny inputs, and invariants the paper states.  CPU only."""
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import BYTES, DNA, Docs, OracleIndex

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(1905_09624)


def rand_dna(n, rng=RNG, alphabet=b"ACGT"):
    return bytes(rng.choice(np.frombuffer(alphabet, np.uint8), size=n))


# ---- hash family: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) -------------

def test_splitmix64_published_outputs():
    # outputs of the reference splitmix64.c started from state 0 and 1234567
    assert oracle.splitmix64(0, 4) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                       0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert oracle.splitmix64(1234567, 5) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_term_hash_uses_ith_seed():
    seeds = oracle.splitmix64(42, 3)
    for i in range(3):
        assert oracle.term_hash(12345, 42, i) == oracle.mix64(12345 ^ seeds[i])


def test_mix64_is_bijective_on_sample():
    xs = RNG.integers(0, 2**63, size=20000, dtype=np.uint64)
    hs = {oracle.mix64(int(x)) for x in xs}
    assert len(hs) == len(set(int(x) for x in xs))


# ---- terms (section 2.1 q-grams, section 2.3 canonical k-mers) --------------

def test_dna_packing_hand_values():
    # A=0 C=1 G=2 T=3, first base most significant
    assert list(oracle.terms(DNA, 4, False, b"ACGT")) == [0 * 64 + 1 * 16 + 2 * 4 + 3]
    assert list(oracle.terms(DNA, 4, False, b"TTTT")) == [255]
    assert list(oracle.terms(DNA, 4, True, b"TTTT")) == [0]       # revcomp AAAA
    assert list(oracle.terms(DNA, 3, False, b"GAT")) == [2 * 16 + 0 + 3]
    # GAT's reverse complement is ATC = 0*16+3*4+1 = 13 < 35
    assert list(oracle.terms(DNA, 3, True, b"GAT")) == [13]
    assert list(oracle.terms(DNA, 3, True, b"gat")) == [13]       # case-insensitive


def test_dna_invalid_windows_skipped():
    t = oracle.terms(DNA, 3, False, b"ACGNACGT")
    # windows ACG, CGN, GNA, NAC, ACG, CGT -> only the three without N
    assert list(t) == [6, 6, 1 * 16 + 2 * 4 + 3]
    assert len(oracle.terms(DNA, 31, True, b"A" * 30)) == 0
    assert len(oracle.terms(DNA, 5, True, b"")) == 0


def test_canonical_equals_reverse_complement():
    comp = bytes.maketrans(b"ACGT", b"TGCA")
    for _ in range(50):
        s = rand_dna(60)
        rc = s.translate(comp)[::-1]
        a = oracle.terms(DNA, 31, True, s)
        b = oracle.terms(DNA, 31, True, rc)
        assert sorted(a) == sorted(b)
        assert np.all(a < 4**31)


def test_bytes_terms_little_endian():
    assert list(oracle.terms(BYTES, 8, False, b"abcdefgh")) == [
        int.from_bytes(b"abcdefgh", "little")]
    assert list(oracle.terms(BYTES, 3, False, b"abcd")) == [
        int.from_bytes(b"abc", "little"), int.from_bytes(b"bcd", "little")]
    assert list(oracle.terms(BYTES, 8, False, b"\xff" * 8)) == [2**64 - 1]


def test_unique_is_a_set():
    a = [5, 3, 5, 1, 3, 3, 2**64 - 1]
    assert list(oracle.unique(a)) == [1, 3, 5, 2**64 - 1]
    assert len(oracle.unique([])) == 0


# ---- closed forms (section 2.1) ---------------------------------------------

def _golden_theorem1():
    for line in open(os.path.join(GOLD, "theorem1_example.txt")):
        if line.strip() and not line.startswith("#"):
            l, p, K, rate, per_million = line.split()
            return int(l), float(p), float(K), float(rate), int(per_million)


def test_theorem1_worked_example():
    l, p, K, printed, per_million = _golden_theorem1()
    f = math.floor(K * l)
    got = oracle.binom_tail_gt(l, p, f)
    assert f"{got:.3g}" == f"{printed:.3g}"               # 0.000143
    assert round(got * 1e6) == per_million
    # independent library evaluation of the same binomial tail
    assert got == pytest.approx(stats.binom.sf(f, l, p), rel=1e-9)


@pytest.mark.parametrize("l", [5, 31, 70, 100, 970])
@pytest.mark.parametrize("p", [0.05, 0.3, 0.5])
def test_theorem1_matches_binomial_sf(l, p):
    for K in (0.0, 0.3, 0.5, 0.8, 1.0):
        f = math.floor(K * l)
        assert oracle.binom_tail_gt(l, p, f) == pytest.approx(
            stats.binom.sf(f, l, p), rel=1e-7, abs=1e-300)


def test_chernoff_bounds_the_exact_tail():
    for l in (10, 70, 300, 2000):
        for p in (0.1, 0.3):
            for K in (p, 0.5, 0.8, 1.0):
                assert oracle.chernoff(l, p, K) >= oracle.binom_tail_gt(l, p, math.floor(K * l))
    l, p, K, _, _ = _golden_theorem1()
    assert oracle.chernoff(l, p, K) == pytest.approx(math.exp(-70 * 0.04 / 1.4))


def test_bloom_fpr_forms():
    # 1 - x <= e^-x makes the exact form >= the exponential one (section 2.1)
    for m in (10, 1000, 10**6):
        for h in (1, 2, 3):
            for n in (1, m // 4, m):
                assert oracle.bloom_fpr(m, h, n) >= oracle.bloom_fpr_exp(m, h, n) - 1e-15
    assert oracle.bloom_fpr(10**6, 1, 10**6) == pytest.approx(1 - math.exp(-1), rel=1e-5)
    # h = 1, n = 1: exactly one bit set, FPR 1/m
    assert oracle.bloom_fpr(64, 1, 1) == pytest.approx(1 / 64)


@pytest.mark.parametrize("h,p,ratio", [(1, 0.3, 2.80367), (3, 0.1, 4.80833), (2, 0.3, 3.5)])
def test_filter_rows_inverts_fpr(h, p, ratio):
    for n in (1, 7, 1000, 123457, 10**6, 8 * 10**6):
        m = oracle.filter_rows(n, h, p)
        # the smallest m whose (exponential-form) FPR is at most p
        assert oracle.bloom_fpr_exp(m, h, n) <= p * (1 + 1e-12)
        assert oracle.bloom_fpr_exp(m - 1, h, n) > p * (1 - 1e-12) or m == 1
    if h != 2:
        assert oracle.filter_rows(10**6, h, p) / 1e6 == pytest.approx(ratio, rel=1e-5)
    assert oracle.filter_rows(0, h, p) == 1


# ---- block plan: Fig. 4 staircase (section 2.2) ------------------------------

def test_fig4_staircase_is_block_maximum():
    steps, curve = [], []
    for line in open(os.path.join(GOLD, "fig4_staircase.txt")):
        if line.startswith("step"):
            _, x, y = line.split()
            steps.append((int(x), float(y)))
        elif line.startswith("curve"):
            _, x, y = line.split()
            curve.append((int(x), float(y)))
    cx = np.array([c[0] for c in curve])
    cy = np.array([c[1] for c in curve])
    # ideal sizes for 100,000 documents by linear interpolation of the curve;
    # sizes are proportional to n for fixed (h, p), so they serve as n
    n = np.round(np.interp(np.arange(100_000), cx, cy) * 1e5).astype(np.uint64)
    perm = RNG.permutation(100_000)
    order, blocks = oracle.plan(n[perm], 8192)
    assert len(blocks) == 13
    assert np.all(np.diff(n[perm][order].astype(np.int64)) >= 0)
    step_vals = sorted({y for _, y in steps if y > 0})
    for b, (first, docs, nmax) in enumerate(blocks):
        last = first + docs - 1
        assert docs == (8192 if b < 12 else 100_000 - 12 * 8192)
        # the block's size is its last (largest) document's
        assert nmax == n[last]
        # the paper's step lies between the curve samples around that document
        lo = cy[cx <= last].max() if np.any(cx <= last) else 0
        hi = cy[cx >= last].min()
        printed = step_vals[b]
        assert lo - 1e-9 <= printed <= hi + 1e-9
        assert nmax / 1e5 == pytest.approx(printed, rel=0.06)


# ---- index and query vs brute force (sections 2.1-2.3) ----------------------

def tiny_docs(n_docs, maxlen, rng, multi=False, alphabet=b"ACGT"):
    docs = []
    for _ in range(n_docs):
        if multi:
            docs.append([rand_dna(int(rng.integers(0, maxlen)), rng, alphabet)
                         for _ in range(int(rng.integers(1, 4)))])
        else:
            docs.append(rand_dna(int(rng.integers(0, maxlen)), rng, alphabet))
    return Docs.from_lists(docs)


CASES = [
    dict(kind=DNA, q=5, canonical=True, h=1, p=0.3, B=0),
    dict(kind=DNA, q=5, canonical=False, h=2, p=0.3, B=3),
    dict(kind=DNA, q=4, canonical=True, h=3, p=0.5, B=1),
    dict(kind=DNA, q=7, canonical=True, h=1, p=0.3, B=7),
    dict(kind=BYTES, q=3, canonical=False, h=2, p=0.2, B=4),
    # the corners of the accepted ranges
    dict(kind=DNA, q=1, canonical=False, h=5, p=0.9, B=2),
    dict(kind=DNA, q=2, canonical=True, h=8, p=0.01, B=0),
    dict(kind=DNA, q=31, canonical=True, h=4, p=0.3, B=3),
    dict(kind=BYTES, q=1, canonical=False, h=8, p=0.5, B=1),
    dict(kind=BYTES, q=8, canonical=False, h=6, p=0.1, B=5),
]


@pytest.mark.parametrize("case", CASES)
def test_index_query_equals_bruteforce(case):
    rng = np.random.default_rng(7 + case["q"] + 10 * case["h"])
    alphabet = b"ACGTN" if case["kind"] == DNA else b"abcdefgh"
    for trial in range(4):
        docs = tiny_docs(int(rng.integers(1, 15)), 120, rng, multi=trial % 2 == 1,
                         alphabet=alphabet)
        ix = OracleIndex(docs, seed=trial * 101, **case)
        for _ in range(4):
            qy = rand_dna(int(rng.integers(0, 60)), rng, alphabet)
            s1, l1 = ix.query_scores(qy)
            s2, l2 = oracle.bruteforce_scores(docs, qy, seed=trial * 101, **case)
            assert l1 == l2
            assert np.array_equal(s1, s2)


def test_matrix_bits_match_definition():
    rng = np.random.default_rng(3)
    docs = tiny_docs(11, 80, rng)
    ix = OracleIndex(docs, kind=DNA, q=5, canonical=True, h=2, p=0.3, B=4, seed=9)
    order = ix.order()
    seeds = oracle.splitmix64(9, 2)
    for b in range(ix.n_blocks):
        blk = ix.block(b)
        assert blk["stride"] % 128 == 0
        want = np.zeros((blk["rows"], blk["stride"]), np.uint8)
        for j in range(blk["docs"]):
            d = order[blk["first"] + j]
            s = docs.bytes[int(docs.str_off[d]):int(docs.str_off[d + 1])].tobytes()
            for t in set(oracle.terms(DNA, 5, True, s).tolist()):
                for i in range(2):
                    r = oracle.mix64(t ^ seeds[i]) % blk["rows"]
                    want[r, j // 8] |= 1 << (j % 8)
        got = ix.matrix()[blk["offset"]:blk["offset"] + blk["rows"] * blk["stride"]]
        assert np.array_equal(got.reshape(want.shape), want)


def test_no_false_negatives_and_exact_limit():
    rng = np.random.default_rng(11)
    docs = tiny_docs(12, 200, rng)
    for p, exact in ((0.3, False), (1e-5, True)):
        ix = OracleIndex(docs, q=7, h=1, p=p, B=5, seed=5, row_align=1)
        for _ in range(10):
            d = int(rng.integers(0, docs.n_docs))
            s = docs.bytes[int(docs.str_off[d]):int(docs.str_off[d + 1])].tobytes()
            a = int(rng.integers(0, max(len(s) - 20, 1)))
            qy = s[a:a + 40] + rand_dna(10, rng)
            sc, l = ix.query_scores(qy)
            ex, l2 = oracle.exact_intersection(docs, qy, q=7)
            assert l == l2
            assert np.all(sc >= ex)
            if exact:
                assert np.array_equal(sc, ex)


def test_compact_with_one_block_equals_classic():
    rng = np.random.default_rng(13)
    docs = tiny_docs(9, 150, rng)
    a = OracleIndex(docs, q=6, h=2, p=0.3, B=0, seed=1)
    b = OracleIndex(docs, q=6, h=2, p=0.3, B=9, seed=1)
    c = OracleIndex(docs, q=6, h=2, p=0.3, B=100, seed=1)
    for _ in range(8):
        qy = rand_dna(50, rng)
        sa, _ = a.query_scores(qy)
        assert np.array_equal(sa, b.query_scores(qy)[0])
        assert np.array_equal(sa, c.query_scores(qy)[0])


def test_permuting_documents_permutes_scores():
    rng = np.random.default_rng(17)
    lists = [rand_dna(int(rng.integers(10, 150)), rng) for _ in range(10)]
    perm = rng.permutation(10)
    a = OracleIndex(Docs.from_lists(lists), q=6, h=1, p=0.3, B=0, seed=3)
    b = OracleIndex(Docs.from_lists([lists[i] for i in perm]), q=6, h=1, p=0.3, B=0, seed=3)
    for _ in range(6):
        qy = rand_dna(60, rng)
        assert np.array_equal(a.query_scores(qy)[0][perm], b.query_scores(qy)[0])


def test_classic_indexes_concatenate():
    # section 2.3: classic indexes with equal parameters concatenate
    rng = np.random.default_rng(19)
    big = rand_dna(300, rng)
    d1 = [big] + [rand_dna(100, rng) for _ in range(7)]
    d2 = [rand_dna(90, rng) for _ in range(5)]
    i1 = OracleIndex(Docs.from_lists(d1), q=5, h=1, p=0.3, B=0, seed=2)
    i2 = OracleIndex(Docs.from_lists(d2 + [big]), q=5, h=1, p=0.3, B=0, seed=2)
    i12 = OracleIndex(Docs.from_lists(d1 + d2), q=5, h=1, p=0.3, B=0, seed=2)
    assert i1.block(0)["rows"] == i2.block(0)["rows"] == i12.block(0)["rows"]
    rows = i12.block(0)["rows"]
    for r in range(0, rows, 7):
        for j in range(len(d1)):
            assert i12.bit(0, r, j) == i1.bit(0, r, j)
        for j in range(len(d2)):
            assert i12.bit(0, r, len(d1) + j) == i2.bit(0, r, j)


# ---- report: threshold and top-k (sections 2.1, 2.2, 2.3) --------------------

def test_report_threshold_and_order():
    sc = np.array([5, 3, 5, 0, 4], np.uint32)
    ids, s = oracle.report(sc, 5, 4, 5, 0)            # T = ceil(4) = 4
    assert list(ids) == [0, 2, 4] and list(s) == [5, 5, 4]
    ids, s = oracle.report(sc, 5, 4, 5, 1)
    assert list(ids) == [0]
    ids, s = oracle.report(sc, 6, 4, 5, 0)            # T = ceil(4.8) = 5
    assert list(ids) == [0, 2]
    ids, s = oracle.report(sc, 0, 0, 1, 0)            # l = 0 reports nothing
    assert len(ids) == 0
    ids, s = oracle.report(sc, 5, 0, 1, 0)            # K = 0: everyone, sorted
    assert list(ids) == [0, 2, 4, 1, 3]
    ids, s = oracle.report(sc, 5, 0, 1, 3)
    assert list(ids) == [0, 2, 4]
    ids, s = oracle.report(sc, 5, 6, 5, 0)            # K > 1: none
    assert len(ids) == 0


# ---- statistics against the closed forms (section 2.1) ----------------------

def _sigma_ok(observed, expected_p, n, k=4.0):
    sd = math.sqrt(expected_p * (1 - expected_p) / n)
    return abs(observed - expected_p) <= k * sd + 1e-12


def test_column_fill_and_term_fpr_match_closed_form():
    rng = np.random.default_rng(23)
    docs = Docs.from_lists([rand_dna(4000, rng) for _ in range(16)])
    for h, p in ((1, 0.3), (3, 0.1)):
        ix = OracleIndex(docs, q=31, h=h, p=p, B=0, seed=77)
        blk = ix.block(0)
        m = blk["rows"]
        mat = ix.matrix().reshape(m, blk["stride"])
        bits = np.unpackbits(mat, axis=1, bitorder="little")[:, :16]
        nt = ix.n_terms()
        for j in range(16):
            fill = bits[:, j].mean()
            want = 1 - (1 - 1 / m) ** (h * int(nt[j]))
            assert _sigma_ok(fill, want, m)
        # random terms: hit rate of one document vs its predicted FPR
        qy = rand_dna(6000, rng)
        sc, l = ix.query_scores(qy)
        for j in range(16):
            want = oracle.bloom_fpr(m, h, int(nt[j]))
            assert _sigma_ok(sc[j] / l, want, l)


def test_short_query_document_fpr_matches_theorem1():
    rng = np.random.default_rng(29)
    docs = Docs.from_lists([rand_dna(3000, rng) for _ in range(40)])
    ix = OracleIndex(docs, q=31, h=1, p=0.3, B=0, seed=5)
    m = ix.block(0)["rows"]
    nt = ix.n_terms()
    l_target, K = 10, (1, 2)   # 10 distinct terms, K = 1/2
    hits, trials, expect = 0, 0, 0.0
    for _ in range(60):
        qy = rand_dna(l_target + 30, rng)
        sc, l = ix.query_scores(qy)
        assert l == l_target
        T = -(-K[0] * l // K[1])
        hits += int(np.sum(sc >= T))
        trials += len(sc)
        for j in range(len(sc)):
            expect += oracle.binom_tail_gt(l, oracle.bloom_fpr(m, 1, int(nt[j])), T - 1)
    rate, want = hits / trials, expect / trials
    assert _sigma_ok(rate, want, trials)


# ---- one document at a time ----------------------------------------------------

def _revcomp(s: bytes) -> bytes:
    return s[::-1].translate(bytes.maketrans(b"ACGT", b"TGCA"))


@pytest.mark.parametrize("kind,q,canonical,h,B", [(DNA, 31, True, 1, 0), (DNA, 11, False, 3, 4),
                                                  (BYTES, 4, False, 2, 0), (BYTES, 8, False, 5, 3)])
def test_doc_scores_equal_index_columns_and_bruteforce(kind, q, canonical, h, B):
    # a document's scores from its own terms at its block's filter size equal
    # its column of the index query and the matrix-free brute force
    rng = np.random.default_rng(50 + q + h)
    mk = (lambda n: rand_dna(n, rng, b"ACGTacgtN")) if kind == DNA else \
        (lambda n: rng.integers(0, 256, n, dtype=np.uint8).tobytes())
    docs = [[mk(int(rng.integers(0, 300))) for _ in range(int(rng.integers(1, 4)))] for _ in range(11)]
    d = Docs.from_lists(docs)
    ix = OracleIndex(d, kind=kind, q=q, canonical=canonical, h=h, p=0.2, B=B, seed=77)
    qs = [mk(int(rng.integers(q, 400))) for _ in range(5)] + [docs[3][0][:150], b""]
    qset = oracle.QuerySet(qs, kind=kind, q=q, canonical=canonical, h=h, p=0.2, seed=77)
    want = [ix.query_scores(x) for x in qs]
    brute = [oracle.bruteforce_scores(d, x, kind=kind, q=q, canonical=canonical, h=h, p=0.2,
                                      B=B, seed=77) for x in qs]
    order = ix.order()
    for b in range(ix.n_blocks):
        blk = ix.block(b)
        for j in range(blk["docs"]):
            doc = int(order[blk["first"] + j])
            got = qset.doc_scores(blk["rows"], docs[doc])
            for k in range(len(qs)):
                assert got[k] == want[k][0][doc] == brute[k][0][doc], (b, doc, k)
    assert list(qset.ell) == [w[1] for w in want]


def test_rc_palindrome_dups_count_every_overlapping_repeat():
    # uniform-random strings with planted reverse-complement palindromes
    # (hairpins): valid windows minus the repeats found = the exact number of
    # distinct canonical q-mers
    rng = np.random.default_rng(31)
    for trial in range(60):
        q = int(rng.choice([31, 31, 25, 21]))   # far repeats improbable at these lengths
        parts = []
        for _ in range(int(rng.integers(1, 6))):
            parts.append(rand_dna(int(rng.integers(0, 400)), rng))
            half = rand_dna(int(rng.integers(q // 2, q + 6)), rng)
            parts.append(half + _revcomp(half))          # palindrome of even length
            if rng.random() < 0.3:
                parts.append(b"N")
        s = b"".join(parts)
        dups, valid = oracle.rc_palindrome_dups(q, s)
        exact = len(oracle.unique(oracle.terms(DNA, q, True, s)))
        assert valid == len(oracle.terms(DNA, q, True, s))
        assert valid - dups == exact, (trial, q, valid, dups, exact)


def test_rc_palindrome_dups_hand_cases():
    half = b"ACGTTGCAAGGCTTACG"                         # 17 bases
    s = half + _revcomp(half)                           # 34: windows 0..3 of 31
    # windows (0, 3) and (1, 2) are reverse complements of each other
    assert oracle.rc_palindrome_dups(31, s) == (2, 4)
    assert oracle.rc_palindrome_dups(31, s[1:33]) == (1, 2)  # the centre pair only
    assert oracle.rc_palindrome_dups(31, s[:32]) == (0, 2)   # off centre: no pair
    assert oracle.rc_palindrome_dups(31, s[:31]) == (0, 1)
    # a repeat far apart is not a palindrome: not counted
    w = rand_dna(31, np.random.default_rng(5))
    far = w + rand_dna(200, np.random.default_rng(6)) + w
    dups, valid = oracle.rc_palindrome_dups(31, far)
    assert dups == 0 and valid - len(oracle.unique(oracle.terms(DNA, 31, True, far))) == 1
