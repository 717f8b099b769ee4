/*
 * cobs.h -- C ABI of the MI355X (gfx950) COBS query library.
 *
 * COBS (Bingmann, Bradley, Gauger, Iqbal, 2019) indexes an ordered collection
 * of documents, each a set of strings, by the q-grams ("terms") of their
 * strings (section 2.1).  Each document gets a Bloom filter; the filters are
 * stored bit-sliced, one row per filter position and one column per document
 * (section 2.2).  The compact variant sorts documents by their number of
 * distinct terms and gives every block of B consecutive documents its own
 * filter size, reducing one large hash modulo each block's size
 * (sections 2.2, 2.3).  A query hashes its distinct terms, gathers the h rows
 * of every term in every block, ANDs them, adds the surviving bits into
 * per-document scores and reports the documents holding at least a fraction
 * K of the query's distinct terms (section 2.2), or the top-k by score.
 *
 * Conventions shared by every call:
 *  - Every call returns a cobs_status; nothing is thrown across the ABI.  On
 *    failure cobs_last_error() (thread-local) describes the cause.
 *  - The caller owns every input buffer.  The library copies what it needs
 *    and keeps no caller pointer after the call returns.
 *  - The library owns every handle and every result array; release them with
 *    the matching *_free call.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls that
 *    return host results synchronise that stream before returning.
 *  - All device memory is HBM of the current HIP device at the time of the
 *    call that creates the object (an offloaded matrix is pinned host
 *    memory); later calls must run on the same device.
 *  - Scores are integers; nothing on the path uses floating point except the
 *    one-time filter sizing on the host.
 *  - Threads: query calls on one index may run at once from several threads
 *    (each takes a workspace of its own from the index's pool).  Calls that
 *    change an index (cobs_tune, cobs_set_tuning, cobs_index_offload,
 *    cobs_index_onload, cobs_index_free) must not overlap any other call on
 *    that index, a running server's included.
 */
#ifndef COBS_H
#define COBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    COBS_OK = 0,
    COBS_EINVAL = 1,      /* malformed argument */
    COBS_ENOMEM = 2,      /* device or host allocation failed */
    COBS_EBUDGET = 3,     /* does not fit a memory budget (serving, out-of-core) */
    COBS_EOVERFLOW = 4,   /* a query's distinct terms exceed the score width */
    COBS_EDEVICE = 5,     /* a HIP runtime call failed */
    COBS_ECANCELLED = 6,  /* the server stopped before the request ran */
    COBS_ESTATE = 7       /* call out of order (e.g. insert before plan) */
} cobs_status;

typedef enum { COBS_TERMS_DNA = 0, COBS_TERMS_BYTES = 1 } cobs_term_kind;
typedef enum { COBS_MEM_HOST = 0, COBS_MEM_DEVICE = 1 } cobs_mem;
typedef enum { COBS_MODE_BATCHED = 0, COBS_MODE_PLAIN = 1 } cobs_mode;

/*
 * Index parameters (sections 2.1-2.3).
 *  kind       COBS_TERMS_DNA: terms are k-mers over A,C,G,T (either case); a
 *             window holding any other byte yields no term; q in 1..31.
 *             COBS_TERMS_BYTES: terms are q consecutive bytes, q in 1..8
 *             (text is one continuous string, section 2.3).
 *  canonical  DNA only: a k-mer and its reverse complement are one term
 *             (section 2.3).
 *  num_hashes h >= 1 hash functions per filter (section 2.1); h <= 8.
 *  fpr        target false-positive rate p of one term lookup, 0 < p < 1.
 *             Block b gets m_b = max(1, ceil(-n_b h / ln(1 - p^(1/h)))) rows,
 *             n_b the largest distinct-term count in the block (the fixed-h
 *             inversion of the Bloom false-positive rate of section 2.1).
 *  block_docs B: 0 builds the classic index (one block, documents in input
 *             order); B > 0 the compact one (documents sorted by (distinct
 *             terms, input id), blocks of B, the last one possibly partial).
 *  seed       hash seed: hash i of term t is mix64(t ^ s_i), s_i the i-th
 *             output of SplitMix64 started at seed; row = hash mod m_b.
 */
typedef struct {
    uint32_t kind;
    uint32_t q;
    uint32_t canonical;
    uint32_t num_hashes;
    double fpr;
    uint32_t block_docs;
    uint32_t reserved;
    uint64_t seed;
} cobs_params;

/*
 * A run of documents.  Document d (0-based within the run) owns strings
 * [doc_str[d], doc_str[d+1]); string s is bytes[str_off[s] .. str_off[s+1]).
 * str_off and doc_str are always host arrays; `bytes` lives in host memory
 * (mem = COBS_MEM_HOST) or in device memory of the current device
 * (mem = COBS_MEM_DEVICE).  Offsets are absolute within `bytes`.
 */
typedef struct {
    const uint8_t *bytes;
    const uint64_t *str_off;
    const uint64_t *doc_str;
    uint32_t n_docs;
    uint32_t mem;
} cobs_docs;

typedef struct cobs_index cobs_index;
typedef struct cobs_builder cobs_builder;
typedef struct cobs_server cobs_server;

/* ---- documents from files (section 2.3) ---------------------------------- */

/*
 * Host-side document collection built from files in the formats the paper
 * reads.  Each call appends documents:
 *  COBS_FORMAT_FASTA        one document; each record ('>' header, then the
 *                           sequence lines, whitespace dropped) is one string,
 *                           so reads are hashed independently; ';' lines are
 *                           comments
 *  COBS_FORMAT_MULTI_FASTA  one document per record (one string each)
 *  COBS_FORMAT_FASTQ        one document; each four-line read ('@' header,
 *                           sequence, '+' line, quality of equal length) is one
 *                           string; EINVAL for a malformed or truncated record
 *                           (nothing of the file is kept)
 *  COBS_FORMAT_TEXT         one document: the whole file as one continuous
 *                           string
 * cobs_docset_view fills a host cobs_docs (for cobs_build or the builder, or
 * as query strings) that stays valid until the next append or the free.
 */
typedef enum {
    COBS_FORMAT_FASTA = 0,
    COBS_FORMAT_MULTI_FASTA = 1,
    COBS_FORMAT_FASTQ = 2,
    COBS_FORMAT_TEXT = 3
} cobs_format;

typedef struct cobs_docset cobs_docset;
cobs_status cobs_docset_create(cobs_docset **out);
cobs_status cobs_docset_add_file(cobs_docset *ds, const char *path, uint32_t format);
cobs_status cobs_docset_add_buffer(cobs_docset *ds, const uint8_t *data, uint64_t len,
                                   uint32_t format);
cobs_status cobs_docset_view(const cobs_docset *ds, cobs_docs *docs);
void cobs_docset_free(cobs_docset *ds);

/* ---- construction (sections 2.1-2.3) ------------------------------------ */

/*
 * Build an index over all documents in one call: distinct-term counts, size
 * sort and block plan, zeroed padded matrix, then one atomic OR per (term,
 * hash).  Rows of block b are rowstride_b bytes, a multiple of 128; bit j of
 * a row (document j of the block) is bit j%8 of byte j/8.  Two builds of the
 * same input give byte-identical matrices.
 * Errors: EINVAL (parameters), ENOMEM, EDEVICE.
 */
cobs_status cobs_build(const cobs_params *params, const cobs_docs *docs,
                       void *stream, cobs_index **out);

/*
 * The same construction in passes, for collections that do not fit one call
 * (documents may be regenerated or streamed between the passes):
 *   create(n_docs) -> count(run, first) for every run -> plan ->
 *   insert(run, first) for every run -> finish.
 * `first` is the collection id of the run's document 0.  Runs may come in any
 * order but must cover every document once per pass, with identical content
 * in both passes.  Out-of-order calls return ESTATE.
 */
cobs_status cobs_builder_create(const cobs_params *params, uint32_t n_docs,
                                void *stream, cobs_builder **out);
cobs_status cobs_builder_count(cobs_builder *b, const cobs_docs *run, uint32_t first);
cobs_status cobs_builder_plan(cobs_builder *b);
cobs_status cobs_builder_insert(cobs_builder *b, const cobs_docs *run, uint32_t first);
cobs_status cobs_builder_finish(cobs_builder *b, cobs_index **out);
void cobs_builder_free(cobs_builder *b);

void cobs_index_free(cobs_index *ix);

typedef struct {
    uint32_t n_docs;
    uint32_t n_blocks;
    cobs_params params;
    uint64_t total_bytes;   /* device bytes of the signature matrix */
    uint64_t score_bytes;   /* device bytes of one query's score buffer: 4 per
                               document, each 8192-document slice rounded up
                               to whole 128-document lanes (the unit by which
                               cobs_serve admits requests) */
    uint32_t host_resident; /* 1 after cobs_index_offload */
    uint32_t n_groups;      /* block groups streamed per batch when offloaded */
    uint64_t stage_bytes;   /* size of each of the two device staging buffers */
} cobs_index_info_t;

cobs_status cobs_index_info(const cobs_index *ix, cobs_index_info_t *info);

/*
 * Out-of-core queries (section 2.3 and section 4: an index need not fit in
 * memory; blocks are read as they are needed).  cobs_index_offload moves the
 * signature matrix into pinned host memory and frees its device memory; every
 * later query batch streams the matrix through two device staging buffers,
 * each of at most device_budget_bytes / 2 and holding a group of whole
 * consecutive blocks: the copy of one group (DMA over the host link) overlaps
 * the gather of the previous one.  A batch therefore reads the whole matrix
 * once over the host link, and large batches amortise it.  A batch whose
 * rows are far fewer than the matrix instead reads each row slice it needs
 * in place, straight from host memory (cobs_host_reads).  Results are
 * identical.  Streamed batches on an offloaded index run one at a time.
 * cobs_index_onload moves the matrix back into device memory.  Neither may
 * run while another thread queries the index.
 * Errors: EBUDGET when half the budget cannot hold the largest block;
 * ESTATE when the matrix already is where it would be moved; ENOMEM; EDEVICE.
 */
cobs_status cobs_index_offload(cobs_index *ix, uint64_t device_budget_bytes);
cobs_status cobs_index_onload(cobs_index *ix);

/*
 * Index files (section 2.3: an index is written once and queried many times,
 * read into memory or as needed).  One file per index, little-endian:
 *   header    "COBSMTX1", header size (u32), kind, q, canonical, num_hashes,
 *             block_docs (u32 each), fpr (f64), seed (u64), n_docs, n_blocks
 *             (u32), total_bytes, matrix offset, metadata FNV-1a 64 (u64)
 *   order     u32[n_docs]   sorted position -> input id
 *   n_terms   u64[n_docs]   distinct terms per input id
 *   blocks    {first u32, docs u32, rows u64, stride u64, offset u64}[n_blocks]
 *   padding   to a multiple of 4096 bytes
 *   matrix    total_bytes: the blocks one after another, each at its offset,
 *             rows of stride bytes, document j of a block at bit j % 8 of
 *             byte j / 8 (the device layout)
 * cobs_index_load checks the magic, the parameters, the checksum, that the
 * order is a permutation and that the block table follows from the stored
 * counts and block sizes (EINVAL otherwise).  device_budget_bytes = 0 puts the matrix in device memory of
 * `device`; otherwise it stays in pinned host memory and queries stream it as
 * after cobs_index_offload with that budget.  The caller owns *out
 * (cobs_index_free).  Errors: EINVAL (I/O, format), EBUDGET, ENOMEM, EDEVICE.
 */
cobs_status cobs_index_save(const cobs_index *ix, const char *path);
cobs_status cobs_index_load(const char *path, int device, uint64_t device_budget_bytes,
                            cobs_index **out);
/*
 * Merge two indexes with identical parameters into a new one (section 2.3:
 * classic indexes with the same parameters concatenate; a compact index is
 * a concatenation of subindices).  The result's documents are a's, then
 * b's with input ids shifted by a's n_docs.  Classic: both must have the
 * same row count; every row is a's row followed by b's.  Compact: a's blocks
 * followed by b's, each keeping its documents and row count (documents are
 * not re-sorted across the two, so the result is the incremental
 * augmentation of a by b).  Every document keeps the score it has in its
 * own index.  Both matrices must be in device memory; the caller owns *out.
 * Errors: EINVAL (parameters, row counts), ESTATE (offloaded input), ENOMEM,
 * EDEVICE.
 */
cobs_status cobs_index_merge(const cobs_index *a, const cobs_index *b, cobs_index **out);
/* Block b: first sorted position, documents, rows m_b, row stride (bytes),
 * byte offset of the block inside the matrix. */
cobs_status cobs_index_block(const cobs_index *ix, uint32_t b, uint32_t *first,
                             uint32_t *docs, uint64_t *rows, uint64_t *stride,
                             uint64_t *offset);
/* order[pos] = input id of the document at sorted position pos (host array
 * of n_docs); distinct-term count per input id into n_terms (may be NULL). */
cobs_status cobs_index_order(const cobs_index *ix, uint32_t *order, uint64_t *n_terms);
/* Copy nbytes of the matrix starting at byte offset into host memory. */
cobs_status cobs_index_read(const cobs_index *ix, uint64_t offset, uint64_t nbytes,
                            void *host_dst);

/* ---- query (section 2.2) ------------------------------------------------ */

/*
 * Options of a query batch.
 *  k_num/k_den  K = k_num / k_den exactly; a document is reported when its
 *               score >= T = ceil(k_num * l / k_den), l the query's distinct
 *               terms; a query with l = 0 reports nothing.  k_den > 0.
 *  topk         0 = every document reaching T; otherwise at most topk of them.
 *  score_bits   16 or 32: the score width of the request; a query with more
 *               than 2^score_bits - 1 distinct terms fails with EOVERFLOW.
 *  mode         COBS_MODE_BATCHED runs the whole batch through one pipeline
 *               (persistent gather kernel); COBS_MODE_PLAIN runs the same
 *               pipeline once per query (one query per launch).
 *  mem          where `bytes` lives (cobs_mem); q_off is always host memory.
 *  chunk        distinct terms per work item of the gather kernel for this
 *               call; 0 = the index's split (see cobs_tuning).  Results
 *               never depend on it.
 */
typedef struct {
    uint32_t k_num;
    uint32_t k_den;
    uint32_t topk;
    uint32_t score_bits;
    uint32_t mode;
    uint32_t mem;
    uint32_t chunk;
} cobs_query_opts;

/* Hits of one query, ordered by (score desc, input id asc). */
typedef struct {
    uint32_t n;           /* reported documents */
    uint32_t num_terms;   /* l = distinct terms of the query */
    uint32_t *doc_id;     /* [n] input ids */
    uint32_t *score;      /* [n] scores */
} cobs_hits;

/*
 * Query n_queries patterns: query i is bytes[q_off[i] .. q_off[i+1]), one
 * string each.  *out receives a library-owned array of n_queries cobs_hits
 * (free with cobs_hits_free(*out, n_queries)).
 * Errors: EINVAL, EOVERFLOW, ENOMEM, EDEVICE.
 */
cobs_status cobs_query_batch(cobs_index *ix, const uint8_t *bytes,
                             const uint64_t *q_off, uint32_t n_queries,
                             const cobs_query_opts *opts, void *stream,
                             cobs_hits **out);

/*
 * Full score vectors: scores[i * n_docs + d] = score of query i for input
 * document d (host array, caller-owned), num_terms[i] = l of query i.  The
 * same gather as cobs_query_batch, without threshold or top-k.
 */
cobs_status cobs_query_scores(cobs_index *ix, const uint8_t *bytes,
                              const uint64_t *q_off, uint32_t n_queries,
                              uint32_t mem, void *stream, uint32_t *scores,
                              uint32_t *num_terms);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * full score vectors as cobs_query_scores, computed without any device
 * allocation.  Every intermediate buffer of the batch (query bytes, terms,
 * hash sets, hashes, plan, tickets, score buffers of split queries) is
 * carved out of one fixed scratch array of 64 MiB that the library holds on
 * each device it runs on until the process ends; a batch that needs more
 * fails with EBUDGET (8 (2 + h) bytes per window, up to 41 more per window
 * of queries longer than 12,288 windows, and 4 bytes per document for every
 * query longer than one work item).
 *  bytes     device memory: query i is bytes[q_off[i] .. q_off[i+1])
 *  q_off     host array [n_queries + 1], non-decreasing
 *  scores    device memory, caller-owned [n_queries * n_docs] u32:
 *            scores[i * n_docs + d] = score of query i for input document d
 *  num_terms device memory [n_queries] u32 (l of each query), or NULL
 * The current device must be the index's; the index must be resident in
 * HBM (not offloaded).  Asynchronous: the work is queued on `stream` and the
 * outputs are valid once it completes.  Every call on one device shares its
 * scratch array, so calls whose work overlaps on the device race (use one
 * stream, or order the streams); the scratch array keeps the last call's
 * contents and each call clears what must start at zero.
 * Errors: EINVAL, EBUDGET, EDEVICE.
 */
cobs_status cobs_query_scores_noalloc(cobs_index *ix, const uint8_t *bytes,
                                      const uint64_t *q_off, uint32_t n_queries,
                                      void *stream, uint32_t *scores,
                                      uint32_t *num_terms);

/*
 * Distinct terms of each query (steps before the gather): terms of query i
 * go to terms[cap_off[i] ..], cap_off[i] = sum over j < i of
 * max(0, len_j - q + 1); num_terms[i] receives l.  The order within a query
 * is unspecified.  Host arrays, caller-owned.
 */
cobs_status cobs_query_terms(const cobs_index *ix, const uint8_t *bytes,
                             const uint64_t *q_off, uint32_t n_queries,
                             uint32_t mem, void *stream, uint64_t *terms,
                             uint32_t *num_terms);

void cobs_hits_free(cobs_hits *hits, uint32_t n);

/*
 * The same query batch as cobs_query_batch with the hits of all queries in
 * one flat, library-owned result object (no per-query allocation).
 */
typedef struct cobs_results cobs_results;
cobs_status cobs_query_results(cobs_index *ix, const uint8_t *bytes, const uint64_t *q_off,
                               uint32_t n_queries, const cobs_query_opts *opts, void *stream,
                               cobs_results **out);
/*
 * Query several indexes as one collection (the paper's tool queries several
 * index files, so that a front-end can pick datasets or categories: section
 * 4, conclusion and future work).  Documents are numbered across the indexes in the given order: input
 * document d of indexes[j] is n_docs(0) + ... + n_docs(j - 1) + d.  The
 * indexes must share the term definition (kind, q, canonical), so each
 * query has the same l, and the same threshold T, in every one; h, p, seed
 * and block size may differ.  Every index runs the batch (opts as in
 * cobs_query_batch) on `stream` in turn; each query's hits over all of them
 * are ordered by (score desc, global id asc), and top-k keeps the topk best
 * over the union.  The result is the query of the compact merge of the
 * indexes (cobs_index_merge), without building it.
 * Errors: EINVAL (NULL or no index, differing kind/q/canonical or device,
 * more than 2^32 - 1 documents in all), and those of cobs_query_batch.
 */
cobs_status cobs_query_multi(cobs_index *const *indexes, uint32_t n_indexes,
                             const uint8_t *bytes, const uint64_t *q_off, uint32_t n_queries,
                             const cobs_query_opts *opts, void *stream, cobs_results **out);

/*
 * View of a result object: query i's hits are doc_id[hit_off[i] .. hit_off[i+1])
 * with score[] alongside, ordered by (score desc, input id asc); num_terms[i]
 * is l.  Pointers stay valid until cobs_results_free.
 */
cobs_status cobs_results_view(const cobs_results *r, uint32_t *n_queries,
                              const uint32_t **num_terms, const uint64_t **hit_off,
                              const uint32_t **doc_id, const uint32_t **score);
void cobs_results_free(cobs_results *r);

/* ---- serving ------------------------------------------------------------ */

/*
 * Continuous-batching server over a resident index.  The server allocates
 * score_budget_bytes of device memory at start as a pool of per-query score
 * buffers (score_bytes of cobs_index_info_t each); a request is admitted, in
 * arrival order, when a buffer is free and holds it until its result is
 * ready.  Admitted requests are grouped into device batches, and up to
 * num_streams batches run on the GPU at once, so requests arriving while
 * others run join the next batch.  Each stream's workspace is sized at start
 * for max_batch_queries queries of max_batch_terms windows in total, so a
 * batch within those limits allocates nothing.
 *  score_budget_bytes  0 = 4096 score buffers, at most 1/4 of the free
 *                      device memory at start
 *  num_streams         concurrent batches in flight (1..8), 0 = 2
 *  max_batch_queries   0 = 4096
 *  max_batch_terms     windows per batch before it is cut, 0 = 2^23 (a
 *                      longer request still runs, as a batch of its own)
 *  score_bits          16 or 32 (0 = 32)
 *  max_inflight        most requests admitted at once (each holds one score
 *                      buffer), 0 = as many as the budget holds; the pool
 *                      holds min(budget / score_bytes, max_inflight) buffers
 */
typedef struct {
    uint64_t score_budget_bytes;
    uint32_t num_streams;
    uint32_t max_batch_queries;
    uint64_t max_batch_terms;
    uint32_t score_bits;
    uint32_t max_inflight;
} cobs_serve_opts;

typedef struct {
    uint64_t submitted, completed, rejected, cancelled, batches;
    uint64_t p50_ns, p99_ns, max_ns;   /* completion - arrival */
    double queries_per_s, lookups_per_s, wall_s;
    uint64_t lookups;
} cobs_serve_stats;

cobs_status cobs_serve(cobs_index *ix, const cobs_serve_opts *opts, cobs_server **out);
/*
 * Submit one query (host bytes, copied).  arrival_ns is the request's arrival
 * on the CLOCK_MONOTONIC clock (0 = now); latency counts from it.  Returns
 * EBUDGET when the budget holds no score buffer at all.
 */
cobs_status cobs_submit(cobs_server *s, const uint8_t *query, uint64_t len,
                        uint32_t k_num, uint32_t k_den, uint32_t topk,
                        uint64_t arrival_ns, uint64_t *ticket);
/* Wait for a ticket; *out receives one library-owned cobs_hits (free with
 * cobs_hits_free(*out, 1)); latency_ns may be NULL. */
cobs_status cobs_wait(cobs_server *s, uint64_t ticket, cobs_hits **out,
                      uint64_t *latency_ns);
/* Drain every admitted request, stop the loop, fill stats, free the server. */
cobs_status cobs_serve_stop(cobs_server *s, cobs_serve_stats *stats);

/*
 * Open-loop load generator for measuring served latency.  A native thread
 * submits query i (bytes[q_off[i] .. q_off[i+1]), host memory) at
 * start + arrival_ns[i], start being the call time plus 1 ms, with that
 * scheduled time as its arrival; the caller's thread waits for every request.
 * latency_ns[i] (completion - scheduled arrival) and n_hits[i] are written
 * when non-NULL; results are released.  Returns the first error.
 */
cobs_status cobs_serve_replay(cobs_server *s, const uint8_t *bytes, const uint64_t *q_off,
                              uint32_t n, const uint64_t *arrival_ns, uint32_t k_num,
                              uint32_t k_den, uint32_t topk, uint64_t *latency_ns,
                              uint32_t *n_hits);

/* ---- tuning --------------------------------------------------------------- */

/*
 * Order in which the gather kernel's persistent wavefronts take the work
 * items (query chunk, column slice).  In both, chunks come in query-size
 * order, largest first.
 *  COBS_ORDER_QUERIES  the slices of one chunk side by side (the grid drains
 *                      evenly over the whole batch);
 *  COBS_ORDER_SLICES   every chunk of one slice before the next slice (the
 *                      slice's rows stay in the last-level cache while the
 *                      batch reads them);
 *  COBS_ORDER_AUTO     slice-major when every slice of the index holds at
 *                      most 128 MiB of rows, else query-major.
 */
typedef enum {
    COBS_ORDER_AUTO = 0,
    COBS_ORDER_QUERIES = 1,
    COBS_ORDER_SLICES = 2,
} cobs_order;

/*
 * How a batch on an offloaded index (cobs_index_offload) reads the matrix
 * in pinned host memory.
 *  COBS_HOST_READS_STREAM    every group of blocks is copied into a device
 *                            staging buffer and gathered there: the whole
 *                            matrix crosses the host link once per batch;
 *  COBS_HOST_READS_IN_PLACE  the gather reads each row slice it needs
 *                            straight from host memory (only the rows of the
 *                            batch's terms cross the link, as random reads);
 *  COBS_HOST_READS_AUTO      in place when the batch's rows (bounded by its
 *                            windows: windows x h x row bytes per term) are
 *                            fewer bytes than the matrix, else streamed.
 */
typedef enum {
    COBS_HOST_READS_AUTO = 0,
    COBS_HOST_READS_STREAM = 1,
    COBS_HOST_READS_IN_PLACE = 2,
} cobs_host_reads;

/*
 * How a batch of one short query (at most 2,048 windows, not offloaded, no
 * full scores) is launched.
 *  COBS_LAUNCH_AUTO    three kernels (terms, set and plan in one workgroup;
 *                      the gather; the hits sorted in one workgroup) and the
 *                      result copy, captured once per launch-shape class as a
 *                      hipGraph and replayed;
 *  COBS_LAUNCH_DIRECT  the general pipeline, every kernel and copy launched on
 *                      the stream.
 */
typedef enum {
    COBS_LAUNCH_AUTO = 0,
    COBS_LAUNCH_DIRECT = 1,
} cobs_launch;

/*
 * Early exit of threshold queries.  A document's score is its count of the
 * query's distinct terms whose rows hold its bit (section 2.2); after c of
 * the l terms it can gain at most l - c more, so once every document of a
 * block's column slice scores below T - (l - c), none of them can be
 * reported.
 *  COBS_PRUNE_OFF  every term is counted for every document (the scoring
 *                  of the paper, which has no pruning);
 *  COBS_PRUNE_ON   a (query, slice) work item holding all of a query's
 *                  terms checks every 64 terms and stops as soon as no
 *                  document of the slice can reach T (not in launches whose
 *                  slices are all at most 512 bytes wide, several terms per
 *                  load).  A batch whose queries are split over several
 *                  items gathers twice: first the leading chunks of every
 *                  query, then the rest, skipping the (query, slice) pairs
 *                  whose merged counts show that no document can reach T.
 *                  Hits, scores and top-k are the same as with
 *                  COBS_PRUNE_OFF: every document that reaches T is counted
 *                  over every term.  Full score vectors (cobs_query_scores)
 *                  and queries with T = 0 are never pruned.
 */
typedef enum {
    COBS_PRUNE_OFF = 0,
    COBS_PRUNE_ON = 1,
} cobs_prune;

/*
 * Launch shape of the gather kernel for an index: `unroll` terms whose rows
 * are in flight per wavefront (h = 1: 4 or 8; h > 1: 2 or 4; a batch of one
 * hash and wide slices with fewer work items than resident wavefronts, a
 * lone short query among them, uses 16 whatever the setting), `chunk`, the
 * most distinct terms per work item (longer queries are split and their
 * counts merged; a batch is split into about two work items per resident
 * wavefront, with items of at most `chunk` terms), `order` (cobs_order),
 * `host_reads` (cobs_host_reads; offloaded indexes only), `launch`
 * (cobs_launch) and `prune` (cobs_prune).  0 = defaults (8 or 2; 16384;
 * COBS_ORDER_AUTO; COBS_HOST_READS_AUTO; COBS_LAUNCH_AUTO; COBS_PRUNE_OFF).
 * Results never depend on any of them.
 */
typedef struct {
    uint32_t unroll;
    uint32_t chunk;
    double gather_ms;    /* cobs_tune: the chosen shape's gather time */
    uint32_t order;
    uint32_t host_reads;
    uint32_t launch;
    uint32_t prune;
} cobs_tuning;

/* Time the gather kernel on the sample batch for every supported unroll and
 * chunk in {default, 512, 1024, 2048, 4096, 8192, 16384, 2^20} in the
 * index's automatic order, then the other order at the fastest pair; keep
 * the fastest shape for this index and report it in *best (order 1 or 2).
 * The sample should resemble the batches to come (a separate query set). */
cobs_status cobs_tune(cobs_index *ix, const uint8_t *bytes, const uint64_t *q_off,
                      uint32_t n_queries, uint32_t mem, void *stream, cobs_tuning *best);
/* Set (or, with zeros, reset) the launch shape explicitly; gather_ms is
 * ignored.  EINVAL: an unroll the index does not support, or an order above
 * COBS_ORDER_SLICES. */
cobs_status cobs_set_tuning(cobs_index *ix, const cobs_tuning *t);

/* ---- device memory ------------------------------------------------------ */

/*
 * Where the library's device memory comes from.  By default every device
 * allocation (matrices, order and slice tables, query workspaces, server
 * score pools, out-of-core staging buffers) is a hipMalloc and is released
 * with hipFree.  A caller that manages device memory itself, such as a
 * framework's caching allocator, installs its own pair here:
 *  alloc(ctx, bytes)  device memory of the current device, at least
 *                     256-byte aligned, or NULL when it cannot (the library
 *                     call then fails with ENOMEM);
 *  free(ctx, ptr)     gives back a pointer alloc returned.  The library waits
 *                     for the device to be idle before it calls free, so
 *                     the memory may be handed out again at once.
 * Both may be called from any thread, server workers included, and must not
 * call into this library.  Every allocation is released through the pair
 * that made it, so the pair and its ctx must stay valid until the last
 * object holding such memory is freed.  Installing a pair affects later
 * allocations only; NULL (or alloc == NULL) restores hipMalloc/hipFree.
 * Pinned host memory (hipHostMalloc) is not routed.
 * Errors: EINVAL when alloc is set and free is not.
 */
typedef struct {
    void *(*alloc)(void *ctx, uint64_t bytes);
    void (*free)(void *ctx, void *ptr);
    void *ctx;
} cobs_allocator;

cobs_status cobs_set_allocator(const cobs_allocator *allocator);

/* ---- measurement -------------------------------------------------------- */

/*
 * Per-kernel timing of the query path: while enabled, every launch of the
 * gather kernel (row gather + AND + ADD + threshold/top-k, the dominant
 * kernel) is bracketed by HIP events recorded on the stream it runs on, and
 * the elapsed times are accumulated.  Process-wide; costs one event pair per
 * launch.  cobs_profile_read copies the totals and, if reset != 0, zeroes them.
 */
typedef struct {
    uint64_t launches;
    double total_ms;
    double last_ms;
    uint64_t row_bytes;   /* algorithmic row bytes of those launches:
                             sum over queries of l * h * (row bytes per term) */
    uint64_t terms;       /* distinct query terms of those launches */
} cobs_kernel_timing;

cobs_status cobs_profile(int enable);

/*
 * Read ceiling of the device: two passes of coalesced, non-temporal 16-byte
 * loads over [buf, buf + bytes) by a persistent grid (each wavefront reading
 * contiguous 64 KiB chunks; the whole grid sweeping the buffer), each timed
 * with HIP events on `stream`; *gbps = bytes / the faster pass's time
 * (10^9 B/s).  The gather kernel's
 * row reads are judged against it beside the HBM peak.  buf: device memory,
 * 16-byte aligned, only read (its contents do not matter); bytes: a positive
 * multiple of 16.  Errors: EINVAL, EDEVICE.
 */
cobs_status cobs_read_bandwidth(const void *buf, uint64_t bytes, void *stream, double *gbps);

/*
 * Read ceiling of random row reads, the access pattern of the gather (section
 * 2.2: one row of the matrix per query term): about `reads` reads of one
 * 1 KiB row each (a wavefront's 64 lanes x 16 bytes, eight rows in flight per
 * wavefront, 8,192 wavefronts), every row drawn uniformly from the
 * floor(bytes / 1024) rows of [buf, buf + bytes) by a counter-based hash.
 * cached != 0: ordinary loads, so that a buffer small enough for the L2 or
 * the last-level cache is read from there; 0: non-temporal loads.  Three
 * passes on `stream`, the first warming the caches; *gbps = bytes read by
 * one pass / the faster of the other two (10^9 B/s).  buf: device memory,
 * 16-byte aligned, only read; bytes: 1 KiB to 2^32 - 1 rows of 1 KiB.
 * Errors: EINVAL, EDEVICE.
 */
cobs_status cobs_read_rows_bandwidth(const void *buf, uint64_t bytes, uint64_t reads, int cached,
                                     void *stream, double *gbps);
cobs_status cobs_profile_read(cobs_kernel_timing *gather, int reset);

/* ---- misc --------------------------------------------------------------- */

const char *cobs_last_error(void);
/* Monotonic clock in ns, the clock cobs_submit's arrival_ns uses. */
uint64_t cobs_now_ns(void);

#ifdef __cplusplus
}
#endif
#endif
