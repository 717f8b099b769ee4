/*
 * Plain, slow CPU oracle of the COBS query path.  TEST INFRASTRUCTURE ONLY:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * call it.  It shares no source with the GPU library.
 *
 * Written for readability against the paper, not for speed: every step is a
 * direct loop over the definition, in the order the paper states it.
 * Parity for the hash values, bit positions and exact score integers is
 * pinned by the tests (brute force, closed forms, invariants), not by the
 * paper, which prints no such values.
 */
#include "cobs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- hashing ------------------------------------------------------------ */

/* SplitMix64 generator step (Steele, Lea, Flood 2014; constants of the
 * published reference implementation). */
uint64_t orc_splitmix64_next(uint64_t *state)
{
    *state += 0x9E3779B97F4A7C15ull;
    return orc_mix64(*state);
}

uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_term_hash(uint64_t term, uint64_t seed, uint32_t i)
{
    /* section 2.1 needs h hash functions; we draw h seeds from SplitMix64 */
    uint64_t st = seed, s = 0;
    for (uint32_t k = 0; k <= i; ++k) s = orc_splitmix64_next(&st);
    return orc_mix64(term ^ s);
}

/* ---- terms (section 2.1 q-grams, section 2.3 canonical k-mers) ---------- */

static int base_code(uint8_t c)
{
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

uint64_t orc_terms(int kind, uint32_t q, int canonical, const uint8_t *s,
                   uint64_t len, uint64_t *out)
{
    uint64_t n = 0;
    if (q == 0 || len < q) return 0;
    for (uint64_t i = 0; i + q <= len; ++i) {
        if (kind == ORC_BYTES) {
            uint64_t t = 0;
            for (uint32_t j = 0; j < q; ++j) t |= (uint64_t)s[i + j] << (8 * j);
            out[n++] = t;
        } else {
            uint64_t fwd = 0, rc = 0;
            int ok = 1;
            for (uint32_t j = 0; j < q; ++j) {
                int c = base_code(s[i + j]);
                if (c < 0) { ok = 0; break; }
                fwd = fwd * 4 + (uint64_t)c;
            }
            if (!ok) continue;
            /* reverse complement: base j from the end, complemented */
            for (uint32_t j = 0; j < q; ++j) {
                int c = base_code(s[i + q - 1 - j]);
                rc = rc * 4 + (uint64_t)(3 - c);
            }
            out[n++] = (canonical && rc < fwd) ? rc : fwd;
        }
    }
    return n;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

uint64_t orc_unique(uint64_t *a, uint64_t n)
{
    if (n == 0) return 0;
    qsort(a, n, sizeof(uint64_t), cmp_u64);
    uint64_t k = 1;
    for (uint64_t i = 1; i < n; ++i)
        if (a[i] != a[k - 1]) a[k++] = a[i];
    return k;
}

/* ---- closed forms (section 2.1) ----------------------------------------- */

uint64_t orc_filter_rows(uint64_t n, uint32_t h, double p)
{
    double m = ceil(-(double)n * (double)h / log(1.0 - pow(p, 1.0 / (double)h)));
    if (!(m >= 1.0)) return 1;
    return (uint64_t)m;
}

double orc_bloom_fpr(double m, uint32_t h, double n)
{
    return pow(1.0 - pow(1.0 - 1.0 / m, (double)h * n), (double)h);
}

double orc_bloom_fpr_exp(double m, uint32_t h, double n)
{
    return pow(1.0 - exp(-(double)h * n / m), (double)h);
}

double orc_binom_tail_gt(uint64_t l, double p, uint64_t f)
{
    /* 1 - sum_{i<=f} C(l,i) p^i (1-p)^(l-i), evaluated as the upper sum */
    if (f >= l) return 0.0;
    if (p <= 0.0) return 0.0;
    if (p >= 1.0) return 1.0;
    double s = 0.0;
    for (uint64_t i = f + 1; i <= l; ++i) {
        double lc = lgamma((double)l + 1) - lgamma((double)i + 1) -
                    lgamma((double)(l - i) + 1);
        s += exp(lc + (double)i * log(p) + (double)(l - i) * log1p(-p));
    }
    return s;
}

double orc_chernoff(uint64_t l, double p, double K)
{
    return exp(-(double)l * (K - p) * (K - p) / (2.0 * (1.0 - p)));
}

/* ---- index construction (sections 2.1-2.3) ------------------------------ */

/* distinct terms of document d, sorted; caller frees */
static uint64_t doc_terms(const orc_params *prm, const uint8_t *bytes,
                          const uint64_t *str_off, const uint64_t *doc_str,
                          uint32_t d, uint64_t **out)
{
    uint64_t total = 0;
    for (uint64_t s = doc_str[d]; s < doc_str[d + 1]; ++s)
        total += str_off[s + 1] - str_off[s];
    uint64_t *t = (uint64_t *)malloc((total + 1) * sizeof(uint64_t));
    uint64_t n = 0;
    for (uint64_t s = doc_str[d]; s < doc_str[d + 1]; ++s)
        n += orc_terms(prm->kind, prm->q, prm->canonical, bytes + str_off[s],
                       str_off[s + 1] - str_off[s], t + n);
    n = orc_unique(t, n);
    *out = t;
    return n;
}

typedef struct { uint64_t n; uint32_t id; } size_key;

static int cmp_size_key(const void *a, const void *b)
{
    const size_key *x = (const size_key *)a, *y = (const size_key *)b;
    if (x->n != y->n) return (x->n > y->n) - (x->n < y->n);
    return (x->id > y->id) - (x->id < y->id);
}

static void hash_seeds(uint64_t seed, uint32_t h, uint64_t *out)
{
    uint64_t st = seed;
    for (uint32_t i = 0; i < h; ++i) out[i] = orc_splitmix64_next(&st);
}

uint32_t orc_plan(const uint64_t *n_terms, uint32_t n_docs, uint32_t B,
                  uint32_t *order, uint32_t *blk_first, uint32_t *blk_docs,
                  uint64_t *blk_nmax)
{
    uint32_t n_blocks;
    if (B == 0) {
        for (uint32_t d = 0; d < n_docs; ++d) order[d] = d;
        n_blocks = n_docs ? 1 : 0;
    } else {
        size_key *k = (size_key *)malloc((n_docs ? n_docs : 1) * sizeof(size_key));
        for (uint32_t d = 0; d < n_docs; ++d) { k[d].n = n_terms[d]; k[d].id = d; }
        qsort(k, n_docs, sizeof(size_key), cmp_size_key);
        for (uint32_t d = 0; d < n_docs; ++d) order[d] = k[d].id;
        free(k);
        n_blocks = (n_docs + B - 1) / B;
    }
    for (uint32_t b = 0; b < n_blocks; ++b) {
        uint32_t first = B ? b * B : 0;
        uint32_t docs = B ? (n_docs - first < B ? n_docs - first : B) : n_docs;
        uint64_t m = 0;   /* the block's largest document sets its filter size */
        for (uint32_t j = 0; j < docs; ++j)
            if (n_terms[order[first + j]] > m) m = n_terms[order[first + j]];
        if (blk_first) blk_first[b] = first;
        if (blk_docs) blk_docs[b] = docs;
        if (blk_nmax) blk_nmax[b] = m;
    }
    return n_blocks;
}

orc_index *orc_build(const orc_params *prm, const uint8_t *bytes,
                     const uint64_t *str_off, const uint64_t *doc_str,
                     uint32_t n_docs)
{
    orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
    ix->prm = *prm;
    ix->n_docs = n_docs;
    ix->hash_seed = (uint64_t *)malloc((prm->h ? prm->h : 1) * sizeof(uint64_t));
    hash_seeds(prm->seed, prm->h, ix->hash_seed);

    /* n_d = |G_q(d)|, exact */
    ix->n_terms = (uint64_t *)malloc((n_docs ? n_docs : 1) * sizeof(uint64_t));
    for (uint32_t d = 0; d < n_docs; ++d) {
        uint64_t *t;
        ix->n_terms[d] = doc_terms(prm, bytes, str_off, doc_str, d, &t);
        free(t);
    }

    /* compact: order by (size, id) and cut blocks of B; classic: one block */
    ix->order = (uint32_t *)malloc((n_docs ? n_docs : 1) * sizeof(uint32_t));
    ix->n_blocks = orc_plan(ix->n_terms, n_docs, prm->B, ix->order, NULL, NULL, NULL);
    uint32_t nb = ix->n_blocks ? ix->n_blocks : 1;
    ix->blk_first = (uint32_t *)calloc(nb, sizeof(uint32_t));
    ix->blk_docs = (uint32_t *)calloc(nb, sizeof(uint32_t));
    ix->blk_rows = (uint64_t *)calloc(nb, sizeof(uint64_t));
    ix->blk_stride = (uint64_t *)calloc(nb, sizeof(uint64_t));
    ix->blk_offset = (uint64_t *)calloc(nb, sizeof(uint64_t));
    uint64_t *nmax = (uint64_t *)calloc(nb, sizeof(uint64_t));
    orc_plan(ix->n_terms, n_docs, prm->B, ix->order, ix->blk_first, ix->blk_docs, nmax);
    uint64_t off = 0;
    for (uint32_t b = 0; b < ix->n_blocks; ++b) {
        uint64_t bytes_per_row = (ix->blk_docs[b] + 7) / 8;
        uint64_t a = prm->row_align ? prm->row_align : 1;
        ix->blk_rows[b] = orc_filter_rows(nmax[b], prm->h, prm->p);
        ix->blk_stride[b] = (bytes_per_row + a - 1) / a * a;
        ix->blk_offset[b] = off;
        off += ix->blk_rows[b] * ix->blk_stride[b];
    }
    free(nmax);
    ix->total_bytes = off;
    ix->bits = (uint8_t *)calloc(off ? off : 1, 1);
    if (!ix->bits) { orc_free(ix); return NULL; }

    /* set bit (row H_i(s) mod m_b, column j) for every term of every document */
    for (uint32_t b = 0; b < ix->n_blocks; ++b) {
        for (uint32_t j = 0; j < ix->blk_docs[b]; ++j) {
            uint32_t d = ix->order[ix->blk_first[b] + j];
            uint64_t *t;
            uint64_t n = doc_terms(prm, bytes, str_off, doc_str, d, &t);
            for (uint64_t x = 0; x < n; ++x) {
                for (uint32_t i = 0; i < prm->h; ++i) {
                    uint64_t row = orc_mix64(t[x] ^ ix->hash_seed[i]) % ix->blk_rows[b];
                    ix->bits[ix->blk_offset[b] + row * ix->blk_stride[b] + j / 8] |=
                        (uint8_t)(1u << (j % 8));
                }
            }
            free(t);
        }
    }
    return ix;
}

void orc_free(orc_index *ix)
{
    if (!ix) return;
    free(ix->hash_seed); free(ix->n_terms); free(ix->order);
    free(ix->blk_first); free(ix->blk_docs); free(ix->blk_rows);
    free(ix->blk_stride); free(ix->blk_offset); free(ix->bits);
    free(ix);
}

int orc_bit(const orc_index *ix, uint32_t b, uint64_t row, uint32_t j)
{
    return (ix->bits[ix->blk_offset[b] + row * ix->blk_stride[b] + j / 8] >> (j % 8)) & 1;
}

/* ---- query (section 2.2) ------------------------------------------------ */

uint64_t orc_query_scores(const orc_index *ix, const uint8_t *query,
                          uint64_t len, uint32_t *scores)
{
    const orc_params *prm = &ix->prm;
    uint64_t *t = (uint64_t *)malloc((len + 1) * sizeof(uint64_t));
    uint64_t l = orc_terms(prm->kind, prm->q, prm->canonical, query, len, t);
    l = orc_unique(t, l);
    memset(scores, 0, ix->n_docs * sizeof(uint32_t));
    uint64_t *rows = (uint64_t *)malloc((prm->h ? prm->h : 1) * sizeof(uint64_t));
    for (uint32_t b = 0; b < ix->n_blocks; ++b) {
        for (uint64_t x = 0; x < l; ++x) {
            for (uint32_t i = 0; i < prm->h; ++i)
                rows[i] = orc_mix64(t[x] ^ ix->hash_seed[i]) % ix->blk_rows[b];
            for (uint32_t j = 0; j < ix->blk_docs[b]; ++j) {
                int all = 1;                     /* AND of the h rows */
                for (uint32_t i = 0; i < prm->h; ++i)
                    all &= orc_bit(ix, b, rows[i], j);
                scores[ix->order[ix->blk_first[b] + j]] += (uint32_t)all;  /* ADD */
            }
        }
    }
    free(rows);
    free(t);
    return l;
}

typedef struct { uint32_t score, id; } hit;

static int cmp_hit(const void *a, const void *b)
{
    const hit *x = (const hit *)a, *y = (const hit *)b;
    if (x->score != y->score) return x->score < y->score ? 1 : -1;
    return (x->id > y->id) - (x->id < y->id);
}

uint32_t orc_report(const uint32_t *scores, uint32_t n_docs, uint64_t l,
                    uint32_t k_num, uint32_t k_den, uint32_t topk,
                    uint32_t *out_id, uint32_t *out_score)
{
    if (l == 0 || k_den == 0) return 0;
    uint64_t T = ((uint64_t)k_num * l + k_den - 1) / k_den;
    hit *h = (hit *)malloc((n_docs ? n_docs : 1) * sizeof(hit));
    uint32_t n = 0;
    for (uint32_t d = 0; d < n_docs; ++d)
        if (scores[d] >= T) { h[n].score = scores[d]; h[n].id = d; ++n; }
    qsort(h, n, sizeof(hit), cmp_hit);
    if (topk && n > topk) n = topk;
    for (uint32_t i = 0; i < n; ++i) { out_id[i] = h[i].id; out_score[i] = h[i].score; }
    free(h);
    return n;
}

/* ---- matrix-free forms -------------------------------------------------- */

static int contains(const uint64_t *a, uint64_t n, uint64_t v)
{
    for (uint64_t i = 0; i < n; ++i) if (a[i] == v) return 1;
    return 0;
}

uint64_t orc_bruteforce_scores(const orc_params *prm, const uint8_t *bytes,
                               const uint64_t *str_off, const uint64_t *doc_str,
                               uint32_t n_docs, const uint8_t *query,
                               uint64_t len, uint32_t *scores)
{
    /* block plan recomputed here from the definition: m_b of the block that
     * holds d after sorting by (size, id) */
    uint64_t *sz = (uint64_t *)malloc((n_docs ? n_docs : 1) * sizeof(uint64_t));
    uint64_t **dt = (uint64_t **)malloc((n_docs ? n_docs : 1) * sizeof(uint64_t *));
    for (uint32_t d = 0; d < n_docs; ++d)
        sz[d] = doc_terms(prm, bytes, str_off, doc_str, d, &dt[d]);
    uint64_t *m_of = (uint64_t *)malloc((n_docs ? n_docs : 1) * sizeof(uint64_t));
    for (uint32_t d = 0; d < n_docs; ++d) {
        /* rank of d in the (size, id) order */
        uint32_t rank = 0;
        for (uint32_t e = 0; e < n_docs; ++e)
            if (sz[e] < sz[d] || (sz[e] == sz[d] && e < d)) ++rank;
        uint64_t nmax = 0;
        for (uint32_t e = 0; e < n_docs; ++e) {
            uint32_t re = 0;
            if (prm->B) {
                for (uint32_t f = 0; f < n_docs; ++f)
                    if (sz[f] < sz[e] || (sz[f] == sz[e] && f < e)) ++re;
                if (re / prm->B != rank / prm->B) continue;
            }
            if (sz[e] > nmax) nmax = sz[e];
        }
        m_of[d] = orc_filter_rows(nmax, prm->h, prm->p);
    }
    uint64_t *qt = (uint64_t *)malloc((len + 1) * sizeof(uint64_t));
    uint64_t l = orc_unique(qt, orc_terms(prm->kind, prm->q, prm->canonical,
                                          query, len, qt));
    uint64_t st = prm->seed;
    uint64_t *seeds = (uint64_t *)malloc((prm->h ? prm->h : 1) * sizeof(uint64_t));
    for (uint32_t i = 0; i < prm->h; ++i) seeds[i] = orc_splitmix64_next(&st);
    for (uint32_t d = 0; d < n_docs; ++d) {
        uint32_t sc = 0;
        for (uint64_t x = 0; x < l; ++x) {
            int all = 1;
            for (uint32_t i = 0; i < prm->h && all; ++i) {
                /* one bit array per filter: bit H_i(s) may be set by any
                 * hash i2 of any term t of the document (section 2.1) */
                uint64_t want = orc_mix64(qt[x] ^ seeds[i]) % m_of[d];
                int any = 0;
                for (uint64_t y = 0; y < sz[d] && !any; ++y)
                    for (uint32_t i2 = 0; i2 < prm->h && !any; ++i2)
                        any = (orc_mix64(dt[d][y] ^ seeds[i2]) % m_of[d]) == want;
                all = any;
            }
            sc += (uint32_t)all;
        }
        scores[d] = sc;
    }
    for (uint32_t d = 0; d < n_docs; ++d) free(dt[d]);
    free(dt); free(sz); free(m_of); free(qt); free(seeds);
    return l;
}

uint64_t orc_exact_intersection(const orc_params *prm, const uint8_t *bytes,
                                const uint64_t *str_off, const uint64_t *doc_str,
                                uint32_t n_docs, const uint8_t *query,
                                uint64_t len, uint32_t *counts)
{
    uint64_t *qt = (uint64_t *)malloc((len + 1) * sizeof(uint64_t));
    uint64_t l = orc_unique(qt, orc_terms(prm->kind, prm->q, prm->canonical,
                                          query, len, qt));
    for (uint32_t d = 0; d < n_docs; ++d) {
        uint64_t *t;
        uint64_t n = doc_terms(prm, bytes, str_off, doc_str, d, &t);
        uint32_t c = 0;
        for (uint64_t x = 0; x < l; ++x) c += (uint32_t)contains(t, n, qt[x]);
        counts[d] = c;
        free(t);
    }
    free(qt);
    return l;
}

/* ---- one document at a time (block and column separability) ------------- */

void orc_term_rows(const orc_params *prm, uint64_t m, const uint64_t *terms,
                   uint64_t n, uint64_t *rows)
{
    uint64_t st = prm->seed;
    for (uint32_t i = 0; i < prm->h; ++i) {
        uint64_t seed_i = orc_splitmix64_next(&st);
        for (uint64_t x = 0; x < n; ++x)
            rows[(uint64_t)i * n + x] = orc_mix64(terms[x] ^ seed_i) % m;
    }
}

void orc_doc_scores(const orc_params *prm, uint64_t m, const uint8_t *bytes,
                    const uint64_t *str_off, uint64_t n_str,
                    const uint64_t *qrows, uint64_t total, const uint64_t *qoff,
                    uint32_t nq, uint32_t *scores)
{
    /* the document's Bloom filter of m bits: bit H_i(t) mod m for every term
     * t of the document and every i < h (section 2.1) */
    uint64_t words = (m + 63) / 64;
    uint64_t *bits = (uint64_t *)calloc(words ? words : 1, sizeof(uint64_t));
    uint64_t longest = 0;
    for (uint64_t k = 0; k < n_str; ++k)
        if (str_off[k + 1] - str_off[k] > longest) longest = str_off[k + 1] - str_off[k];
    uint64_t *t = (uint64_t *)malloc((longest + 1) * sizeof(uint64_t));
    uint64_t *seeds = (uint64_t *)malloc((prm->h ? prm->h : 1) * sizeof(uint64_t));
    hash_seeds(prm->seed, prm->h, seeds);
    for (uint64_t k = 0; k < n_str; ++k) {
        uint64_t n = orc_terms(prm->kind, prm->q, prm->canonical, bytes + str_off[k],
                               str_off[k + 1] - str_off[k], t);
        for (uint64_t x = 0; x < n; ++x)
            for (uint32_t i = 0; i < prm->h; ++i) {
                uint64_t r = orc_mix64(t[x] ^ seeds[i]) % m;
                bits[r / 64] |= 1ull << (r % 64);
            }
    }
    /* score: query terms whose h bits are all set */
    for (uint32_t k = 0; k < nq; ++k) {
        uint32_t c = 0;
        for (uint64_t x = qoff[k]; x < qoff[k + 1]; ++x) {
            int all = 1;
            for (uint32_t i = 0; i < prm->h; ++i) {
                uint64_t r = qrows[(uint64_t)i * total + x];
                all &= (int)((bits[r / 64] >> (r % 64)) & 1u);
            }
            c += (uint32_t)all;
        }
        scores[k] = c;
    }
    free(bits); free(t); free(seeds);
}

static int cmp_u64_plain(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

uint64_t orc_rc_palindrome_dups(uint32_t q, const uint8_t *s, uint64_t len,
                                uint64_t *valid_windows)
{
    signed char *c = (signed char *)malloc(len ? len : 1);
    uint64_t valid = 0, run = 0;
    for (uint64_t x = 0; x < len; ++x) {
        c[x] = (signed char)base_code(s[x]);
        run = c[x] < 0 ? 0 : run + 1;
        if (q && run >= q) ++valid;
    }
    if (valid_windows) *valid_windows = valid;
    if (q == 0 || q > 31 || len < q) { free(c); return 0; }
    uint64_t cap = 64, n = 0;
    uint64_t *dup = (uint64_t *)malloc(cap * sizeof(uint64_t));
    /* a window pair needs an arm of at least k = (q + 2) / 2 (at most 16).
     * Filter: A = the k bases ending at p, s[p] least significant; B = the
     * complements of the k bases from p + 1, s[p+1] least significant; the
     * arm reaches k exactly when A == B and those 2k bases are ACGT. */
    const uint32_t k = (q + 2) / 2;
    const uint64_t mask = k >= 32 ? ~0ull : (1ull << (2 * k)) - 1;
    uint64_t A = 0, B = 0;
    int64_t last_bad = -1;   /* last non-ACGT position among those read */
    for (uint64_t x = 0; x < len && x < k; ++x) {   /* B for p = -1: bases 0 .. k-1 */
        int y = c[x];
        if (y < 0) { last_bad = (int64_t)x; y = 0; }
        B |= (uint64_t)(3 - y) << (2 * x);
    }
    for (uint64_t p = 0; p + 1 < len; ++p) {
        int y = c[p] < 0 ? 0 : c[p];
        A = ((A << 2) | (uint64_t)y) & mask;
        /* B: drop base p, read base p + k */
        B >>= 2;
        if (p + k < len) {
            int z = c[p + k];
            if (z < 0) { last_bad = (int64_t)(p + k); z = 0; }
            B |= (uint64_t)(3 - z) << (2 * (k - 1));
        } else {
            break;   /* no arm of k bases fits any more */
        }
        if (p + 1 < k || A != B || last_bad >= (int64_t)(p + 1 - k)) continue;
        /* arm: the longest a with s[p-j] the complement of s[p+1+j], j < a */
        uint64_t a = 0;
        while (a <= p && p + 1 + a < len) {
            int u = c[p - a], v = c[p + 1 + a];
            if (u < 0 || v < 0 || u + v != 3) break;
            ++a;
        }
        /* the palindrome [p+1-h2, p+h2] of length q + d = 2 h2 holds window
         * i = p+1-h2 and window j = i+d, the reverse complement of window i */
        for (uint64_t h2 = k; h2 <= a; ++h2) {
            uint64_t i = p + 1 - h2, d = 2 * h2 - q;
            if (n == cap) { cap *= 2; dup = (uint64_t *)realloc(dup, cap * sizeof(uint64_t)); }
            dup[n++] = i + d;
        }
    }
    qsort(dup, n, sizeof(uint64_t), cmp_u64_plain);
    uint64_t cnt = 0;
    for (uint64_t x = 0; x < n; ++x)
        if (x == 0 || dup[x] != dup[x - 1]) ++cnt;
    free(dup);
    free(c);
    return cnt;
}

/* ---- accessors ---------------------------------------------------------- */

uint32_t orc_n_blocks(const orc_index *ix) { return ix->n_blocks; }

void orc_block_info(const orc_index *ix, uint32_t b, uint32_t *first,
                    uint32_t *docs, uint64_t *rows, uint64_t *stride,
                    uint64_t *offset)
{
    *first = ix->blk_first[b];
    *docs = ix->blk_docs[b];
    *rows = ix->blk_rows[b];
    *stride = ix->blk_stride[b];
    *offset = ix->blk_offset[b];
}

const uint32_t *orc_order(const orc_index *ix) { return ix->order; }
const uint64_t *orc_n_terms(const orc_index *ix) { return ix->n_terms; }
const uint8_t *orc_bits(const orc_index *ix) { return ix->bits; }
uint64_t orc_total_bytes(const orc_index *ix) { return ix->total_bytes; }
