/*
 * Plain, slow CPU oracle of the COBS query path (Bingmann, Bradley, Gauger,
 * Iqbal: "COBS: a Compact Bit-Sliced Signature Index", 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the GPU library.
 *
 * Every function follows the paper's definitions directly:
 *   terms          -- q-grams of each string of a document (section 2.1);
 *                     optional canonical k-mers (section 2.3)
 *   bloom filters  -- h hash functions, set bit h_i(s) for every term
 *                     (section 2.1); one-sided error
 *   sizing         -- the fixed-h inversion of the Bloom false-positive
 *                     formula of section 2.1: m = -n h / ln(1 - p^(1/h))
 *   compact layout -- documents sorted by size, one classic sub-index per
 *                     B consecutive documents, one hash reduced modulo each
 *                     block's filter size (sections 2.2 and 2.3)
 *   query          -- hash the query terms, AND the h rows per term, ADD the
 *                     indicator vectors into per-document scores, keep the
 *                     documents reaching K * |G_q(P)| (section 2.2)
 *   closed forms   -- Bloom FPR (section 2.1), Theorem 1 binomial tail and
 *                     its Chernoff bound (section 2.1)
 */
#ifndef COBS_ORACLE_H
#define COBS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DNA = 0, ORC_BYTES = 1 };

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): one step of the generator. */
uint64_t orc_splitmix64_next(uint64_t *state);
/* The SplitMix64 output finaliser applied to x. */
uint64_t orc_mix64(uint64_t x);
/* i-th hash of a term: mix64(term ^ seed_i), seed_i = i-th SplitMix64 output
 * of the generator started at `seed`. */
uint64_t orc_term_hash(uint64_t term, uint64_t seed, uint32_t i);

/* All q-gram windows of one string, in window order, duplicates kept.
 * DNA: ACGT (either case) -> 0..3, first base most significant; a window
 * holding any other byte is skipped; canonical -> min(forward, revcomp).
 * BYTES: q <= 8 bytes, little-endian, zero extended.
 * Returns the number of terms written to out (capacity >= len). */
uint64_t orc_terms(int kind, uint32_t q, int canonical, const uint8_t *s,
                   uint64_t len, uint64_t *out);
/* Sort ascending and remove duplicates in place; returns the new length. */
uint64_t orc_unique(uint64_t *a, uint64_t n);

/* Filter rows for n distinct terms: max(1, ceil(-n h / ln(1 - p^(1/h)))). */
uint64_t orc_filter_rows(uint64_t n, uint32_t h, double p);

/* Closed forms (section 2.1). */
double orc_bloom_fpr(double m, uint32_t h, double n);      /* (1-(1-1/m)^(hn))^h */
double orc_bloom_fpr_exp(double m, uint32_t h, double n);  /* (1-e^(-hn/m))^h */
/* Theorem 1: Pr[X > f], X ~ Binomial(l, p), summed over the upper tail. */
double orc_binom_tail_gt(uint64_t l, double p, uint64_t f);
/* Chernoff bound exp(-l (K-p)^2 / (2(1-p))), valid for K >= p. */
double orc_chernoff(uint64_t l, double p, double K);

typedef struct {
    int kind;            /* ORC_DNA or ORC_BYTES */
    uint32_t q;          /* term length */
    int canonical;       /* DNA only */
    uint32_t h;          /* hash functions */
    double p;            /* target false-positive rate */
    uint32_t B;          /* documents per block; 0 = classic (one block, no reorder) */
    uint64_t seed;       /* hash seed */
    uint32_t row_align;  /* row stride alignment in bytes (power of two) */
} orc_params;

typedef struct {
    orc_params prm;
    uint32_t n_docs, n_blocks;
    uint64_t *hash_seed;     /* [h] */
    uint64_t *n_terms;       /* [n_docs] distinct terms per original document */
    uint32_t *order;         /* [n_docs] sorted position -> original id */
    uint32_t *blk_first;     /* [n_blocks] first sorted position */
    uint32_t *blk_docs;      /* [n_blocks] documents in block */
    uint64_t *blk_rows;      /* [n_blocks] m_b */
    uint64_t *blk_stride;    /* [n_blocks] bytes per row */
    uint64_t *blk_offset;    /* [n_blocks] byte offset of the block */
    uint64_t total_bytes;
    uint8_t *bits;           /* the bit-sliced signature matrix */
} orc_index;

/* Block plan (sections 2.2, 2.3): B = 0 keeps input order in one block; else
 * order by (n_terms asc, id asc) and cut blocks of B.  Fills order[n_docs]
 * and, when non-NULL, per-block first position, size and largest n_terms.
 * Returns the number of blocks. */
uint32_t orc_plan(const uint64_t *n_terms, uint32_t n_docs, uint32_t B,
                  uint32_t *order, uint32_t *blk_first, uint32_t *blk_docs,
                  uint64_t *blk_nmax);
/* Documents: doc d owns strings [doc_str[d], doc_str[d+1]); string i is
 * bytes[str_off[i] .. str_off[i+1]). */
orc_index *orc_build(const orc_params *prm, const uint8_t *bytes,
                     const uint64_t *str_off, const uint64_t *doc_str,
                     uint32_t n_docs);
void orc_free(orc_index *ix);
/* Read bit (block, row, column j) of the matrix. */
int orc_bit(const orc_index *ix, uint32_t block, uint64_t row, uint32_t j);

/* Score one query string against every document: scores[original id].
 * Returns l = |G_q(P)| (distinct terms). */
uint64_t orc_query_scores(const orc_index *ix, const uint8_t *query,
                          uint64_t len, uint32_t *scores);

/* Threshold T = ceil(k_num * l / k_den); keep score >= T (none when l = 0),
 * order by (score desc, original id asc), keep the first topk (0 = all).
 * Writes up to n_docs pairs; returns the number kept. */
uint32_t orc_report(const uint32_t *scores, uint32_t n_docs, uint64_t l,
                    uint32_t k_num, uint32_t k_den, uint32_t topk,
                    uint32_t *out_id, uint32_t *out_score);

/* Matrix-free definition: score(d) = #{s in G(P): for all i exists t in G(d)
 * and i2 with H_i2(t) mod m_b(d) = H_i(s) mod m_b(d)}.  Recomputes the block plan
 * itself.  For tiny inputs only. */
uint64_t orc_bruteforce_scores(const orc_params *prm, const uint8_t *bytes,
                               const uint64_t *str_off, const uint64_t *doc_str,
                               uint32_t n_docs, const uint8_t *query,
                               uint64_t len, uint32_t *scores);
/* Exact q-gram set intersection |G(P) cap G(d)| for every document. */
uint64_t orc_exact_intersection(const orc_params *prm, const uint8_t *bytes,
                                const uint64_t *str_off, const uint64_t *doc_str,
                                uint32_t n_docs, const uint8_t *query,
                                uint64_t len, uint32_t *counts);

/* Block and column separability (section 2.2): a document's score depends
 * only on its own terms, its block's filter size m and the query, so large
 * collections are checked one document at a time.
 * orc_term_rows: rows[i * n + x] = H_i(terms[x]) mod m for i < h.
 * orc_doc_scores: the document made of strings [str_off[k], str_off[k+1])
 * of bytes, k < n_str, as a Bloom filter of m bits (bit H_i(t) mod m for
 * every term t and i < h); scores[k] = number of query terms x in
 * [qoff[k], qoff[k+1]) whose h rows qrows[i * total + x] are all set.  The
 * query terms must be each query's distinct terms G(P). */
void orc_term_rows(const orc_params *prm, uint64_t m, const uint64_t *terms,
                   uint64_t n, uint64_t *rows);
void orc_doc_scores(const orc_params *prm, uint64_t m, const uint8_t *bytes,
                    const uint64_t *str_off, uint64_t n_str,
                    const uint64_t *qrows, uint64_t total, const uint64_t *qoff,
                    uint32_t nq, uint32_t *scores);

/* DNA string, canonical q-mers: windows j whose term equals that of an
 * earlier window i of the same string through a reverse-complement
 * palindrome covering both (window j is the reverse complement of window i;
 * the windows overlap when j - i < q).  These are the only repeats a
 * uniform-random string is likely to hold at this length (a hairpin of q + 1
 * bases around a centre); repeats through a periodic stretch or between
 * unrelated positions are not found.  *valid_windows: windows without a
 * non-ACGT byte.  Returns the number of such windows j. */
uint64_t orc_rc_palindrome_dups(uint32_t q, const uint8_t *s, uint64_t len,
                                uint64_t *valid_windows);

/* Accessors used by the Python wrapper. */
uint32_t orc_n_blocks(const orc_index *ix);
void orc_block_info(const orc_index *ix, uint32_t b, uint32_t *first,
                    uint32_t *docs, uint64_t *rows, uint64_t *stride,
                    uint64_t *offset);
const uint32_t *orc_order(const orc_index *ix);
const uint64_t *orc_n_terms(const orc_index *ix);
const uint8_t *orc_bits(const orc_index *ix);
uint64_t orc_total_bytes(const orc_index *ix);

#ifdef __cplusplus
}
#endif
#endif
