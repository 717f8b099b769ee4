// Device-side data layouts and kernel launchers of the COBS query library.
// Host code (lib.cpp, serve.cpp) calls only these launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cobs {

constexpr int kMaxHashes = 8;
constexpr uint64_t kInvalidTerm = ~0ull;   // DNA window with a non-ACGT byte
constexpr uint32_t kSliceBytes = 1024;     // one wavefront: 64 lanes x 16 bytes
constexpr uint32_t kLdsTableSlots = 16384; // largest dedup table held in LDS (128 KiB)
constexpr uint32_t kLdsTinySlots = 2048;   // 16 KiB tables: many workgroups per CU
// Queries of up to kLdsMaxWindows windows dedup in LDS: a table of twice
// their windows rounded up to a power of two, at most kLdsTableSlots (load
// at most 0.75); longer queries use a table in device memory.
constexpr uint64_t kLdsMaxWindows = 12288;
constexpr uint32_t kSortRun = 2048;        // candidates sorted in LDS per run
constexpr uint32_t kSliceDocs = 8192;      // documents per slice (score buffer stride)
constexpr uint32_t kDedupWindowsPerGroup = 16384; // windows per workgroup of a global-table query
constexpr uint32_t kDefaultChunkCap = 16384;      // largest automatic work item (terms)

struct Seeds {
    uint64_t s[kMaxHashes];
};

struct TermSpec {
    uint32_t kind;       // 0 DNA, 1 BYTES
    uint32_t q;
    uint32_t canonical;
    uint32_t h;
};

// One wavefront-wide column slice of one block: up to 8192 documents.
struct SliceDesc {
    uint64_t base;     // byte offset of (row 0, first byte of the slice)
    uint32_t stride;   // row stride of the block in bytes
    uint32_t rows;     // m_b
    uint32_t width;    // bytes of the slice (multiple of 16, <= 1024)
    uint32_t ndocs;    // documents in the slice
    uint32_t doc0;     // sorted position of the slice's first document
    uint32_t block;
    uint32_t acc_off;  // first word of the slice in a query's score buffer
    uint32_t lanes;    // lanes holding documents: ceil(ndocs / 128)
};

// Score buffer of one query (split queries only): for each slice, 128 * lanes
// words from acc_off on; n_docs + 127 * n_slices words at most.

// Per-query state filled by the plan kernel.
struct QInfo {
    uint64_t hbase;    // first unique term of the query in the term arrays
    uint32_t ell;      // distinct terms
    uint32_t nch;      // term chunks
    uint32_t pbase;    // score-buffer slot (queries split into several chunks)
    uint32_t thr;      // T = ceil(k_num * ell / k_den); > ell means none
};

// Per-string descriptor used by the build kernels.
struct StrDesc {
    uint64_t byte_off;   // offset of the string in the byte buffer
    uint64_t wbase;      // first window of the string in the run
    uint32_t doc;        // document index within the piece
    uint32_t pad;
};

// Per-document placement used by the insert kernel.
struct DocPos {
    uint64_t block_off;  // byte offset of the block
    uint32_t rows;
    uint32_t stride;
    uint32_t col;        // column (position within the block)
    uint32_t pad;
};

struct GatherArgs {
    const uint8_t *matrix;
    const SliceDesc *slices;
    const uint32_t *order;
    const uint64_t *hashes;
    const QInfo *qinfo;
    const uint32_t *qorder;            // [n_queries] work order of the queries
    const uint32_t *chunk_prefix;      // [n_queries + 1], in qorder order
    unsigned long long *work_counter;  // device scalar, zero at launch; items = chunks x n_slices
    uint32_t *tickets;                 // [n_queries * n_slices], zero; left zero by every launch
    uint32_t *accum;                   // score buffers of split queries (zero between launches)
    uint64_t acc_words;                // words per score buffer
    unsigned long long *cand_counter;  // device scalar
    uint64_t *cand_key;                // (score << 32) | ~input_id
    uint32_t *cand_q;
    uint32_t *qcount;                  // [n_queries] candidates per query
    uint32_t *full_scores;             // optional [n_queries * n_docs]
    uint64_t cand_cap;
    uint32_t n_queries, n_slices, h, chunk, topk, n_docs;
    // item order: 0 = query-major (the slices of one chunk side by side,
    // chunks in qorder order); 1 = slice-major (every chunk of one slice, in
    // qorder order, before the next slice)
    uint32_t slice_major;
    // 1: documents that can no longer reach their query's threshold stop
    // being counted (never with full_scores)
    uint32_t prune;
    // split queries under pruning run in two launches: 0 = one launch (every
    // chunk); 1 = the first ceil(nch * f) chunks of every query, f =
    // phase1_f0 + phase1_fz / sqrt(l) (all of them when f >= 0.9), whose
    // last one marks dead[q * n_slices + slice] when no document of the
    // slice can reach T; 2 = the remaining chunks (a dead slice's skip their
    // terms; the last chunk clears the mark)
    uint32_t phase;
    float phase1_f0, phase1_fz;
    uint32_t *dead;                    // [n_queries * n_slices], zero; left zero after phase 2
};

// ---- query path ----------------------------------------------------------

// Term extraction: one term per window of every query (kInvalidTerm for DNA windows with
// a non-ACGT byte).  qstart[i]: first byte of query i; wbase[i]: first window;
// the windows end at wbase[n_queries] (device), total_windows bounds it from
// above and sets the grid.
// bytes: 4-byte aligned, with 64 readable bytes after the last query.
// Also zeroes nterms[0, n_queries).
hipError_t launch_extract(const uint8_t *bytes, const uint64_t *qstart, const uint64_t *wbase,
                          uint32_t n_queries, uint64_t total_windows, TermSpec ts,
                          uint64_t *terms, uint32_t *nterms, hipStream_t st);

// Per-query set of terms (hash-set dedup) and the h hashes of each
// distinct term; nterms[i] = l of query i (zeroed by launch_extract).  A query
// whose set fits in LDS is one workgroup with an LDS table: lds_q lists the
// n_tiny queries with dedup_tiny_table(windows), then n_small others with
// dedup_small_table(windows), then n_large others.  A larger one (listed in
// g_q) has dedup_table_slots(windows) global slots at table + tbase[i]
// (cleared here) and dedup_groups(windows) workgroups of kDedupWindowsPerGroup
// windows; its windows are partitioned by hash into LDS sets, or, when a
// partition is too large for one, share a device table;
// gprefix[j]: first workgroup of g_q[j], g_groups = gprefix[n_g];
// table_slots: total global slots.
hipError_t launch_dedup(const uint64_t *terms, const uint64_t *wbase, const uint64_t *tbase,
                        const uint32_t *lds_q, uint32_t n_tiny, uint32_t n_small, uint32_t n_large,
                        const uint32_t *g_q, const uint32_t *gprefix, uint32_t n_g,
                        uint32_t g_groups, uint64_t *table, uint64_t table_slots,
                        uint64_t *uterms, uint64_t *hashes, uint32_t *nterms, TermSpec ts,
                        Seeds seeds, hipStream_t st);
bool dedup_tiny_table(uint64_t windows);       // LDS table of kLdsTinySlots slots or fewer
bool dedup_small_table(uint64_t windows);      // LDS table of kLdsTableSlots / 2 slots or fewer
uint64_t dedup_table_cap(uint64_t windows);    // hash-set capacity for a query (power of 2)
uint64_t dedup_table_slots(uint64_t windows);  // global slots (0: one LDS table)
uint32_t dedup_groups(uint64_t windows);       // workgroups of the query
// Per-query chunks, thresholds, score-buffer slots, work totals; zeroes
// counters.
// qorder: the queries by size class, largest first (work items follow that
// order); chunk_prefix[i]: first chunk of query qorder[i].  A query split
// into several chunks uses score buffer slot[i] when slot is non-NULL, else
// the next free one in query order.
hipError_t launch_plan(const uint32_t *nterms, const uint64_t *wbase, const uint32_t *slot,
                       uint32_t n_queries, uint32_t chunk, uint32_t n_slices, uint32_t k_num,
                       uint32_t k_den, uint64_t ell_limit, QInfo *qinfo, uint32_t *qorder,
                       uint32_t *chunk_prefix, uint64_t *total_items,
                       unsigned long long *work_counter, unsigned long long *cand_counter,
                       uint32_t *qcount, uint32_t *flags, hipStream_t st);

// The persistent gather / AND / ADD / threshold-or-top-k kernel.
// planes: counter planes (>= bits of the largest l); unroll: terms whose rows
// are in flight per wavefront (h = 1: 4 or 8; h > 1: 2 or 4).  packed: every
// slice of a.slices is at most kPackedSliceBytes wide, and 2, 4 or 8 terms
// share one load (64 / G lanes each, G from the slice's width).
constexpr uint32_t kPackedSliceBytes = 512;
hipError_t launch_gather(const GatherArgs &a, int planes, int unroll, int grid, bool packed,
                         hipStream_t st);
int gather_planes_for(uint64_t max_terms);        // instantiated plane count to use
int gather_default_unroll(int h);
bool gather_unroll_valid(int unroll, int h);
int gather_grid(int planes, int unroll, int h, bool packed);   // persistent grid: CUs x resident blocks

// Hit ordering: group candidates by query and sort each query's segment by
// (score desc, input id asc); write the first min(count, topk) hits.
hipError_t launch_group_sort(const uint64_t *cand_key, const uint32_t *cand_q,
                             const unsigned long long *n_cand, uint64_t cap,
                             uint32_t n_queries, uint32_t topk,
                             const uint32_t *qcount, uint32_t *qstart, uint32_t *qcursor,
                             uint64_t *seg_a, uint64_t *seg_b, uint32_t *out_start,
                             uint32_t *out_n, uint32_t *out_id, uint32_t *out_score,
                             hipStream_t st);

// A batch of one query of at most max_windows <= kLdsMaxWindows windows: terms, set, hashes and the plan in one workgroup (terms straight into an LDS
// set); the same outputs as launch_extract + launch_dedup + launch_plan with
// n_queries = 1.  bytes: the query, 4-byte aligned, 64 readable bytes after.
hipError_t launch_front_one(const uint8_t *bytes, const uint64_t *wbase, uint64_t max_windows,
                            const uint32_t *slot, uint64_t *uterms, uint64_t *hashes,
                            uint32_t *nterms, TermSpec ts, Seeds seeds, uint32_t chunk,
                            uint32_t n_slices, uint32_t k_num, uint32_t k_den, uint64_t ell_limit,
                            QInfo *qinfo, uint32_t *qorder, uint32_t *chunk_prefix,
                            uint64_t *total_items, unsigned long long *work_counter,
                            unsigned long long *cand_counter, uint32_t *qcount, uint32_t *flags,
                            hipStream_t st);
// The hits of a batch of one query, sorted in place in cand_key (tmp: as
// many keys of scratch): out_start[0..1], out_n[0], out_id, out_score as
// launch_group_sort writes them for n_queries = 1; the first inline_cap of
// them also to inline_id and inline_score.
hipError_t launch_sort_one(uint64_t *cand_key, uint64_t *tmp, const unsigned long long *n_cand,
                           uint64_t cap, uint32_t topk, uint32_t *out_start, uint32_t *out_n,
                           uint32_t *out_id, uint32_t *out_score, uint32_t *inline_id,
                           uint32_t *inline_score, uint32_t inline_cap, hipStream_t st);

// ---- construction ------------------------------------------------------------

hipError_t launch_count(const uint8_t *bytes, const StrDesc *strs, uint32_t n_strs,
                        uint64_t total_windows, const uint64_t *tbase, const uint32_t *tlog2,
                        uint64_t *table, uint32_t *empty_flag, unsigned long long *counts,
                        TermSpec ts, hipStream_t st);

hipError_t launch_insert(const uint8_t *bytes, const StrDesc *strs, uint32_t n_strs,
                         uint64_t total_windows, const DocPos *pos, uint32_t *matrix,
                         TermSpec ts, Seeds seeds, hipStream_t st);

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st);

// Scratch memory of the allocation-free query entry point: one file-scope
// device array of kScratchBytes, loaded with the library on every device it
// runs on and held until the process ends.  scratch_address gives its address
// on the current device (looked up once per device with
// hipGetSymbolAddress); host code passes that address to kernels, never the
// array's host-side name.
constexpr uint64_t kScratchBytes = 64ull << 20;
hipError_t scratch_address(void **ptr);

// One read pass over bytes / 16 16-byte words at p (16-byte aligned) by
// kReadGrid workgroups of 256 threads; pattern 0: per-wavefront chunks of
// kReadChunk words, 1: grid-wide sweep.  sink: kReadGrid words, written only
// in the improbable case that keeps the loads alive.
constexpr uint32_t kReadGrid = 2048;
constexpr uint64_t kReadChunk = 4096;
hipError_t launch_read(const void *p, uint64_t bytes, int pattern, uint32_t *sink, hipStream_t st);
// Random row reads: each of the kReadGrid * 4 wavefronts reads per_wave
// (a multiple of 8) rows of kSliceBytes drawn from the bytes / kSliceBytes
// rows at p (rows < 2^32), with ordinary (cached) or non-temporal loads.
hipError_t launch_read_rows(const void *p, uint64_t bytes, uint64_t per_wave, bool cached,
                            uint64_t seed, uint32_t *sink, hipStream_t st);

// Classic merge: every row of out (out_stride bytes) = the na document bits
// of a's row, then b's row bits; strides are multiples of 4.
hipError_t launch_concat_rows(const uint8_t *a, uint64_t a_stride, uint32_t na, const uint8_t *b,
                              uint64_t b_stride, uint8_t *out, uint64_t out_stride, uint64_t rows,
                              hipStream_t st);

}  // namespace cobs
