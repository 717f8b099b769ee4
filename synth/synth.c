/*
 * Seeded synthetic inputs for the COBS workloads: random-ACGT documents and
 * DNA queries (planted substrings with substitutions, or random), Zipf text
 * documents and text queries.  Holds no part of the index or query method.
 *
 * Every random number is a Philox4x32-10 output (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC 2011) addressed by a
 * counter (index, sub-index, stream) under a 64-bit key, so any document
 * byte or query byte can be regenerated anywhere in O(1), on the host or on
 * the device (synth_dev.hip implements the same bases generator).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

enum {
    ST_DOC_LEN = 1, ST_DOC_BASES = 2, ST_Q_LEN = 3, ST_Q_PICK = 4,
    ST_Q_SUBST = 5, ST_Q_BASES = 6, ST_VOC = 7, ST_WORDS = 8, ST_TQ = 9,
    ST_TQ_BYTES = 10, ST_ARRIVAL = 11,
};

void synth_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0, p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t stream, uint64_t idx, uint32_t sub, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), sub, stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    synth_philox(ctr, key, out);
}

static uint64_t u64_of(const uint32_t o[4], int w) { return (uint64_t)o[w] | ((uint64_t)o[w + 1] << 32); }
static double unit53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }
/* uniform integer in [lo, hi] */
static uint64_t uniform_int(uint64_t x, uint64_t lo, uint64_t hi)
{
    unsigned __int128 r = (unsigned __int128)x * (unsigned __int128)(hi - lo + 1);
    return lo + (uint64_t)(r >> 64);
}
static double normal01(const uint32_t o[4])
{
    double u1 = ((double)(u64_of(o, 0) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    double u2 = unit53(u64_of(o, 2));
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* ---- DNA ---------------------------------------------------------------- */

static const char ACGT[4] = {'A', 'C', 'G', 'T'};

/* base i of document d */
static inline uint8_t doc_base(uint64_t seed, uint32_t d, uint64_t i)
{
    uint32_t o[4];
    draw(seed, ST_DOC_BASES, i >> 6, d, o);
    uint32_t w = o[(i >> 4) & 3];
    return (uint8_t)ACGT[(w >> (2 * (i & 15))) & 3];
}

/* bases [from, from+n) of document d; 64 bases per Philox call */
void synth_doc_bases(uint64_t seed, uint32_t d, uint64_t from, uint64_t n, uint8_t *out)
{
    uint64_t i = from, end = from + n;
    while (i < end) {
        uint32_t o[4];
        draw(seed, ST_DOC_BASES, i >> 6, d, o);
        uint64_t stop = ((i >> 6) + 1) << 6;
        if (stop > end) stop = end;
        for (; i < stop; ++i) {
            uint32_t w = o[(i >> 4) & 3];
            *out++ = (uint8_t)ACGT[(w >> (2 * (i & 15))) & 3];
        }
    }
}

/* Document lengths.  kind 0: uniform length in [a, b];
 * kind 1: distinct-31-mer target uniform in [a, b], length target + 30;
 * kind 2: target min(cap, round(exp(N(ln median, sigma)))), length target+30. */
void synth_doc_lengths(uint64_t seed, int kind, uint32_t n_docs, double a, double b,
                       double sigma, double cap, uint32_t q, uint64_t *len)
{
    for (uint32_t d = 0; d < n_docs; ++d) {
        uint32_t o[4];
        draw(seed, ST_DOC_LEN, d, 0, o);
        if (kind == 0) {
            len[d] = uniform_int(u64_of(o, 0), (uint64_t)a, (uint64_t)b);
        } else if (kind == 1) {
            len[d] = uniform_int(u64_of(o, 0), (uint64_t)a, (uint64_t)b) + (q - 1);
        } else {
            double t = round(exp(log(a) + sigma * normal01(o)));
            if (t > cap) t = cap;
            len[d] = (uint64_t)t + (q - 1);
        }
    }
}

/* DNA query i.  Length: kind 0 fixed a; kind 1 floor(exp(U(ln a, ln b))).
 * Planted (even i when planted_every == 2, never when 0): a random document
 * at least as long as the query (up to 64 tries, else the query is random),
 * a uniform offset, each base substituted with probability subst by one of
 * the other three.  Random: uniform bases.  Returns the length; when out is
 * NULL only the length is computed.  *src receives the source document or
 * -1, *off the offset. */
uint64_t synth_dna_query(uint64_t seed, uint32_t i, int len_kind, double a, double b,
                         int planted_every, double subst, uint32_t n_docs,
                         const uint64_t *doc_len, uint8_t *out, int64_t *src,
                         uint64_t *off)
{
    uint32_t o[4];
    draw(seed, ST_Q_LEN, i, 0, o);
    uint64_t L = len_kind == 0 ? (uint64_t)a
                               : (uint64_t)floor(exp(log(a) + unit53(u64_of(o, 0)) * (log(b) - log(a))));
    int64_t s = -1;
    uint64_t offset = 0;
    if (planted_every && (i % (uint32_t)planted_every) == 0 && n_docs) {
        for (uint32_t t = 0; t < 64; ++t) {
            draw(seed, ST_Q_PICK, i, t, o);
            uint32_t d = (uint32_t)uniform_int(u64_of(o, 0), 0, n_docs - 1);
            if (doc_len[d] >= L) {
                s = d;
                offset = uniform_int(u64_of(o, 2), 0, doc_len[d] - L);
                break;
            }
        }
    }
    if (src) *src = s;
    if (off) *off = offset;
    if (!out) return L;
    if (s >= 0) {
        synth_doc_bases(seed, (uint32_t)s, offset, L, out);
        /* one draw per 4 bases: 16-bit fraction for the substitution test,
         * 16 bits for the choice among the 3 other bases */
        const uint32_t cut = (uint32_t)(subst * 65536.0 + 0.5);
        for (uint64_t j = 0; j < L; ++j) {
            if ((j & 3) == 0) draw(seed, ST_Q_SUBST, j >> 2, i, o);
            const uint32_t wv = o[j & 3];
            if ((wv & 0xFFFFu) < cut) {
                int c = out[j] == 'A' ? 0 : out[j] == 'C' ? 1 : out[j] == 'G' ? 2 : 3;
                int r = (int)(((wv >> 16) * 3u) >> 16);  /* 0..2 */
                out[j] = (uint8_t)ACGT[(c + 1 + r) & 3];
            }
        }
    } else {
        for (uint64_t j = 0; j < L; j += 64) {
            draw(seed, ST_Q_BASES, j >> 6, i, o);
            for (uint64_t k = j; k < L && k < j + 64; ++k)
                out[k] = (uint8_t)ACGT[(o[(k >> 4) & 3] >> (2 * (k & 15))) & 3];
        }
    }
    return L;
}

/* ---- text --------------------------------------------------------------- */

/* Vocabulary word w: length uniform in [lmin, lmax], uniform bytes. */
uint32_t synth_word(uint64_t seed, uint32_t w, uint32_t lmin, uint32_t lmax, uint8_t *out)
{
    uint32_t o[4];
    draw(seed, ST_VOC, w, 0, o);
    uint32_t L = (uint32_t)uniform_int(u64_of(o, 0), lmin, lmax);
    for (uint32_t j = 0; j < L; j += 16) {
        draw(seed, ST_VOC, w, 1 + j / 16, o);
        for (uint32_t k = j; k < L && k < j + 16; ++k)
            out[k] = (uint8_t)(o[(k - j) / 4] >> (8 * ((k - j) % 4)));
    }
    return L;
}

/* Zipf(s) cumulative weights over ranks 1..V (cdf[V-1] == 1). */
void synth_zipf_cdf(uint32_t V, double s, double *cdf)
{
    double acc = 0;
    for (uint32_t r = 0; r < V; ++r) { acc += pow((double)(r + 1), -s); cdf[r] = acc; }
    for (uint32_t r = 0; r < V; ++r) cdf[r] /= acc;
}

static uint32_t zipf_pick(const double *cdf, uint32_t V, double u)
{
    uint32_t lo = 0, hi = V - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* Text document d of exactly len bytes: Zipf-ranked vocabulary words, each
 * followed by one space, the last word cut at len.  words/wlen hold the
 * vocabulary (word w at words + w*wmax). */
void synth_text_doc(uint64_t seed, uint32_t d, uint64_t len, const double *cdf, uint32_t V,
                    const uint8_t *words, const uint32_t *wlen, uint32_t wmax, uint8_t *out)
{
    uint64_t pos = 0, k = 0;
    uint32_t o[4];
    while (pos < len) {
        if ((k & 1) == 0) draw(seed, ST_WORDS, k >> 1, d, o);
        double u = unit53(u64_of(o, (k & 1) ? 2 : 0));
        uint32_t w = zipf_pick(cdf, V, u);
        for (uint32_t j = 0; j < wlen[w] && pos < len; ++j) out[pos++] = words[(uint64_t)w * wmax + j];
        if (pos < len) out[pos++] = ' ';
        ++k;
    }
}

/* Text document lengths: round(exp(N(ln median, sigma))), at least min, at most cap. */
void synth_text_lengths(uint64_t seed, uint32_t n_docs, double median, double sigma,
                        double lo, double cap, uint64_t *len)
{
    for (uint32_t d = 0; d < n_docs; ++d) {
        uint32_t o[4];
        draw(seed, ST_DOC_LEN, d, 0, o);
        double t = round(exp(log(median) + sigma * normal01(o)));
        if (t > cap) t = cap;
        if (t < lo) t = lo;
        len[d] = (uint64_t)t;
    }
}

/* Text query i: length uniform in [a, b]; even i planted (exact substring of
 * a random document at least that long, bytes replaced with probability
 * subst by a different uniform byte), odd i uniform random bytes.  The
 * planted bytes are read from docs (doc d at docs + doc_off[d]). */
uint64_t synth_text_query(uint64_t seed, uint32_t i, uint64_t a, uint64_t b, double subst,
                          uint32_t n_docs, const uint64_t *doc_off, const uint8_t *docs,
                          uint8_t *out, int64_t *src)
{
    uint32_t o[4];
    draw(seed, ST_TQ, i, 0, o);
    uint64_t L = uniform_int(u64_of(o, 0), a, b);
    int64_t s = -1;
    uint64_t offset = 0;
    if ((i & 1) == 0 && n_docs) {
        for (uint32_t t = 0; t < 64; ++t) {
            draw(seed, ST_TQ, i, 1 + t, o);
            uint32_t d = (uint32_t)uniform_int(u64_of(o, 0), 0, n_docs - 1);
            uint64_t dl = doc_off[d + 1] - doc_off[d];
            if (dl >= L) { s = d; offset = uniform_int(u64_of(o, 2), 0, dl - L); break; }
        }
    }
    if (src) *src = s;
    if (!out) return L;
    if (s >= 0) {
        memcpy(out, docs + doc_off[s] + offset, L);
        for (uint64_t j = 0; j < L; ++j) {
            draw(seed, ST_TQ_BYTES, j, i, o);
            if ((double)o[0] * (1.0 / 4294967296.0) < subst)
                out[j] = (uint8_t)(out[j] + 1 + (uint8_t)(((uint64_t)o[1] * 255u) >> 32));
        }
    } else {
        for (uint64_t j = 0; j < L; j += 16) {
            draw(seed, ST_TQ_BYTES, j >> 4, 0x80000000u | i, o);
            for (uint64_t k = j; k < L && k < j + 16; ++k)
                out[k] = (uint8_t)(o[(k - j) / 4] >> (8 * ((k - j) % 4)));
        }
    }
    return L;
}

/* Poisson arrival times (seconds) at `rate`: cumulative exponential gaps. */
void synth_arrivals(uint64_t seed, uint32_t n, double rate, uint32_t tag, double *t)
{
    double acc = 0;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t o[4];
        draw(seed, ST_ARRIVAL, i, tag, o);
        double u = ((double)(u64_of(o, 0) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
        acc += -log(u) / rate;
        t[i] = acc;
    }
}

/* Uniform double in [0,1) from (stream, idx, sub): for tests of the generator. */
double synth_uniform(uint64_t seed, uint32_t stream, uint64_t idx, uint32_t sub)
{
    uint32_t o[4];
    draw(seed, stream, idx, sub, o);
    return unit53(u64_of(o, 0));
}

/* Single base, for tests. */
uint8_t synth_doc_base(uint64_t seed, uint32_t d, uint64_t i) { return doc_base(seed, d, i); }
