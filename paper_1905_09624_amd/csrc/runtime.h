// Host runtime of the COBS library: device buffers, the resident index and
// the query-batch pipeline shared by cobs_query_batch and the server.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/cobs.h"
#include "kernels.h"

namespace cobs {

cobs_status set_error(cobs_status st, const std::string &msg);
cobs_status hip_error(hipError_t e, const char *what);

#define COBS_HIP(call)                                            \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::cobs::hip_error(e_, #call); \
    } while (0)

// grow-only device buffer
// Device memory of the library: hipMalloc/hipFree, or the allocator the
// caller installed with cobs_set_allocator when the memory was allocated.
hipError_t dev_alloc(void **p, size_t bytes);
void dev_free(void *p);
template <typename T> hipError_t dev_alloc(T **p, size_t bytes)
{
    return dev_alloc(reinterpret_cast<void **>(p), bytes);
}

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release();
    hipError_t ensure(size_t bytes, bool zero = false, hipStream_t st = nullptr);
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// grow-only pinned host buffer
struct HostBuf {
    void *p = nullptr;
    size_t cap = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() { release(); }
    void release();
    hipError_t ensure(size_t bytes);
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

struct Block {
    uint32_t first, docs;
    uint64_t rows, stride, offset, nmax;
};

// Everything one query batch needs on the device; reused across batches.
struct Workspace {
    DevBuf bytes, meta, terms, uterms, hashes, table, head;
    DevBuf tickets, qinfo, qorder, chunk_prefix, accum;
    DevBuf cand_key, cand_q, qcount, gstart, gcursor, seg_a, seg_b, counters;
    DevBuf out_id, out_score, full;
    HostBuf h_stage, h_small, h_out;
    uint64_t tickets_slots = 0;
    uint64_t accum_words = 0;
    uint64_t cand_cap = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};   // gather timing (cobs_profile)
    // Captured launch sequences of single short queries (run_batch), one per
    // launch-shape class, replayed with hipGraphLaunch; each remembers the
    // buffer addresses it was captured with.
    struct Graph {
        std::vector<uint64_t> key;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;
    hipStream_t capture = nullptr;   // private stream the sequences are captured on
    bool graphs_broken = false;      // capture failed once: direct launches only
    ~Workspace();
};

// Host view of a query batch's results.
struct BatchOut {
    std::vector<uint32_t> num_terms;   // l per query
    std::vector<uint32_t> n;           // hits per query
    std::vector<uint32_t> start;       // first hit per query
    const uint32_t *ids = nullptr;     // pinned, valid until the next batch
    const uint32_t *scores = nullptr;
    double gather_ms = 0;              // when BatchSpec::time_gather
};

struct BatchSpec {
    const uint8_t *bytes = nullptr;
    const uint64_t *q_off = nullptr;
    uint32_t n = 0;
    uint32_t mem = COBS_MEM_HOST;
    uint32_t k_num = 0, k_den = 1, topk = 0, score_bits = 32;
    uint32_t chunk = 0;                // terms per work item; 0 = automatic
    uint32_t chunk_cap = 0;            // automatic chunk's maximum; 0 = tuned or kDefaultChunkCap
    uint32_t unroll = 0;               // terms in flight per wavefront; 0 = tuned or default
    uint32_t order = 0;                // cobs_order of the work items; 0 = tuned or by slice size
    uint32_t host_reads = 0;           // cobs_host_reads (offloaded index); 0 = tuned or automatic
    int prune = -1;                    // cobs_prune; -1 = the index's setting
    uint32_t *full_scores = nullptr;   // host [n * n_docs]: full score mode
    uint64_t *terms_out = nullptr;     // host [windows]: terms-only mode
    const uint32_t *slots = nullptr;   // host [n]: score-buffer slot of each query in accum
    uint32_t *accum = nullptr;         // device score buffers (zero); NULL = the workspace's
    bool time_gather = false;          // HIP events around the gather launch
};

}  // namespace cobs

struct cobs_index {
    cobs_params prm{};
    int device = 0;
    uint32_t n_docs = 0;
    std::vector<cobs::Block> blocks;
    std::vector<uint32_t> order;       // sorted position -> input id
    std::vector<uint64_t> n_terms;     // per input id
    std::vector<cobs::SliceDesc> slices;
    uint8_t *d_matrix = nullptr;
    uint64_t total_bytes = 0;
    uint32_t *d_order = nullptr;
    cobs::SliceDesc *d_slices = nullptr;
    // every slice is at most kPackedSliceBytes wide: the matrix in HBM is
    // gathered by the packed kernel (several terms per load)
    bool packed = false;
    cobs::Seeds seeds{};
    int tuned_unroll = 0;              // set by cobs_tune (0 = default)
    uint32_t tuned_chunk = 0;          // set by cobs_tune (0 = automatic)
    uint32_t tuned_order = 0;          // set by cobs_tune (0 = by slice size)
    uint64_t acc_words = 0;            // words of one query's score buffer
    std::mutex pool_mu;
    std::vector<cobs::Workspace *> pool;

    // Out-of-core residency (cobs_index_offload): the matrix in pinned host
    // memory, streamed group by group (whole blocks) through two device
    // staging buffers; one streamed batch at a time.
    struct Group {
        uint32_t slice0, n_slices;   // slices of the group's blocks
        uint64_t off, bytes;         // byte range of the matrix
    };
    uint8_t *h_matrix = nullptr;
    uint8_t *h_dev_matrix = nullptr;   // device address of h_matrix (rows read in place)
    uint32_t tuned_host_reads = 0;     // cobs_tuning.host_reads
    uint32_t tuned_launch = 0;         // cobs_tuning.launch
    uint32_t tuned_prune = 0;          // cobs_tuning.prune
    std::vector<Group> groups;
    cobs::SliceDesc *d_group_slices = nullptr;   // slices, base relative to their group
    uint8_t *d_stage[2] = {nullptr, nullptr};
    uint64_t stage_bytes = 0;
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_copy[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
    std::mutex stream_mu;

    void release_offload();
    ~cobs_index();
};

namespace cobs {

// Shared helpers of the host runtime (lib.cpp).
cobs_status check_params(const cobs_params *p);
TermSpec term_spec(const cobs_params &p);
// Index layout for the order already in ix and these block sizes: row counts,
// strides, offsets, slices and score-buffer offsets (host only).
cobs_status layout_blocks(cobs_index *ix, const std::vector<uint32_t> &block_docs);
// The layout a build gives: compact order by (distinct terms, input id), blocks of B.
cobs_status make_layout(cobs_index *ix);
// Device copies of the order and the slice table.
cobs_status upload_layout(cobs_index *ix, hipStream_t st);

Workspace *acquire_workspace(cobs_index *ix);
void release_workspace(cobs_index *ix, Workspace *ws);

// Run one query batch end to end on stream st (synchronises st).
cobs_status run_batch(cobs_index *ix, Workspace &ws, const BatchSpec &b, hipStream_t st,
                      BatchOut &out);

// Grow every buffer of ws for batches of up to max_queries queries holding
// max_windows windows in total, so that such batches allocate nothing.
cobs_status reserve_workspace(cobs_index *ix, Workspace &ws, uint64_t max_windows,
                              uint32_t max_queries, hipStream_t st);

// Fill library-owned cobs_hits from a BatchOut (queries [q0, q0+n)).
cobs_status make_hits(const BatchOut &o, uint32_t q0, uint32_t n, cobs_hits *dst);

uint64_t now_ns();

}  // namespace cobs
