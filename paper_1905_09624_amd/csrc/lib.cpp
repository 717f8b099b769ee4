// COBS library: errors, device buffers, construction and the resident index
// (the query path is in query.cpp; offload, files and merging in
// index_ops.cpp).
//
// Construction follows sections 2.1-2.3 of the COBS paper: exact distinct
// q-gram counts per document, documents sorted by (count, input id) and cut
// into blocks of B (classic: one block in input order), per-block filter size
// m_b = max(1, ceil(-n_b h / ln(1 - p^(1/h)))), rows padded to 128 bytes,
// one atomic OR per (term, hash).  The query path is section 2.2: hash the
// query's distinct terms, gather and AND the h rows per term, ADD into
// per-document scores, keep score >= ceil(K l) or the top-k.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <ctime>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "runtime.h"

namespace cobs {

static thread_local std::string g_err;

cobs_status set_error(cobs_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

cobs_status hip_error(hipError_t e, const char *what)
{
    const cobs_status st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
                               ? COBS_ENOMEM : COBS_EDEVICE;
    (void)hipGetLastError();
    return set_error(st, std::string(what) + ": " + hipGetErrorString(e));
}

uint64_t now_ns()
{
    timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (uint64_t)t.tv_sec * 1000000000ull + (uint64_t)t.tv_nsec;
}

namespace {

std::mutex g_alloc_mu;
cobs_allocator g_alloc{};                                  // alloc == NULL: hipMalloc
std::unordered_map<void *, cobs_allocator> g_alloc_owner;   // caller-allocated pointers

}  // namespace

hipError_t dev_alloc(void **p, size_t bytes)
{
    cobs_allocator a;
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        a = g_alloc;
    }
    if (!a.alloc) {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) *p = nullptr;
        return e;
    }
    void *q = a.alloc(a.ctx, bytes);
    *p = q;
    if (!q) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_alloc_owner[q] = a;
    return hipSuccess;
}

void dev_free(void *p)
{
    if (!p) return;
    cobs_allocator a{};
    bool owned = false;
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        auto it = g_alloc_owner.find(p);
        if (it != g_alloc_owner.end()) {
            a = it->second;
            owned = true;
            g_alloc_owner.erase(it);
        }
    }
    if (!owned) {
        (void)hipFree(p);
        return;
    }
    // hipFree waits for the device; a caller's allocator may hand the memory
    // out again at once, so wait here for the work that still reads it
    (void)hipDeviceSynchronize();
    a.free(a.ctx, p);
}

void DevBuf::release()
{
    dev_free(p);
    p = nullptr;
    cap = 0;
}

hipError_t DevBuf::ensure(size_t bytes, bool zero, hipStream_t st)
{
    if (bytes <= cap && p) return hipSuccess;
    release();
    size_t want = bytes < 256 ? 256 : bytes + bytes / 4;
    want = (want + 255) & ~size_t(255);
    hipError_t e = dev_alloc(&p, want);
    if (e != hipSuccess) return e;
    cap = want;
    if (zero) return hipMemsetAsync(p, 0, want, st);
    return hipSuccess;
}

void HostBuf::release()
{
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
}

hipError_t HostBuf::ensure(size_t bytes)
{
    if (bytes <= cap && p) return hipSuccess;
    release();
    size_t want = bytes < 4096 ? 4096 : bytes + bytes / 4;
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    cap = want;
    return hipSuccess;
}

Workspace::~Workspace()
{
    for (hipEvent_t &e : ev)
        if (e) (void)hipEventDestroy(e);
    for (Graph &g : graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (capture) (void)hipStreamDestroy(capture);
}

cobs_status check_params(const cobs_params *p)
{
    if (!p) return set_error(COBS_EINVAL, "params is NULL");
    if (p->kind == COBS_TERMS_DNA) {
        if (p->q < 1 || p->q > 31) return set_error(COBS_EINVAL, "DNA q must be in 1..31");
    } else if (p->kind == COBS_TERMS_BYTES) {
        if (p->q < 1 || p->q > 8) return set_error(COBS_EINVAL, "BYTES q must be in 1..8");
    } else {
        return set_error(COBS_EINVAL, "unknown term kind");
    }
    if (p->num_hashes < 1 || p->num_hashes > (uint32_t)kMaxHashes)
        return set_error(COBS_EINVAL, "num_hashes must be in 1..8");
    if (!(p->fpr > 0.0 && p->fpr < 1.0)) return set_error(COBS_EINVAL, "fpr must be in (0,1)");
    return COBS_OK;
}

static Seeds make_seeds(uint64_t seed)
{
    // SplitMix64 (Steele, Lea, Flood 2014): seed_i is its i-th output
    Seeds s{};
    uint64_t st = seed;
    for (int i = 0; i < kMaxHashes; ++i) {
        st += 0x9E3779B97F4A7C15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        s.s[i] = z ^ (z >> 31);
    }
    return s;
}

TermSpec term_spec(const cobs_params &p)
{
    TermSpec t;
    t.kind = p.kind;
    t.q = p.q;
    t.canonical = p.kind == COBS_TERMS_DNA ? (p.canonical ? 1u : 0u) : 0u;
    t.h = p.num_hashes;
    return t;
}

// Bloom filter rows for n distinct terms: the fixed-h inversion of the
// false-positive rate (1 - e^(-hn/m))^h = p (section 2.1)
static uint64_t filter_rows(uint64_t n, uint32_t h, double p)
{
    const double m = std::ceil(-(double)n * (double)h / std::log(1.0 - std::pow(p, 1.0 / (double)h)));
    if (!(m >= 1.0)) return 1;
    return (uint64_t)m;
}

}  // namespace cobs

using namespace cobs;

void cobs_index::release_offload()
{
    for (int i = 0; i < 2; ++i) {
        dev_free(d_stage[i]);
        if (ev_copy[i]) (void)hipEventDestroy(ev_copy[i]);
        if (ev_done[i]) (void)hipEventDestroy(ev_done[i]);
        d_stage[i] = nullptr;
        ev_copy[i] = ev_done[i] = nullptr;
    }
    if (copy_stream) (void)hipStreamDestroy(copy_stream);
    dev_free(d_group_slices);
    if (h_matrix) (void)hipHostFree(h_matrix);
    copy_stream = nullptr;
    d_group_slices = nullptr;
    h_matrix = nullptr;
    h_dev_matrix = nullptr;
    groups.clear();
    stage_bytes = 0;
}

cobs_index::~cobs_index()
{
    for (Workspace *w : pool) delete w;
    release_offload();
    dev_free(d_matrix);
    dev_free(d_order);
    dev_free(d_slices);
}

// ---- construction -------------------------------------------------------------

struct cobs_builder {
    cobs_params prm{};
    uint32_t n_docs = 0;
    hipStream_t st = nullptr;
    int device = 0;
    int state = 0;   // 0 counting, 1 planned (inserting), 2 finished
    std::vector<uint64_t> n_terms;
    std::vector<uint8_t> counted, inserted;
    std::vector<uint32_t> rank;   // input id -> sorted position
    cobs_index *ix = nullptr;
    DevBuf bytes, strs, tbase, tlog2, table, eflag, counts, pos;
    ~cobs_builder() { delete ix; }
};

namespace {

constexpr uint64_t kPieceWindows = 1ull << 27;

struct Piece {
    uint32_t d0, d1;   // documents of the run
};

cobs_status check_run(const cobs_builder *b, const cobs_docs *run, uint32_t first)
{
    if (!run) return set_error(COBS_EINVAL, "docs is NULL");
    if ((uint64_t)first + run->n_docs > b->n_docs)
        return set_error(COBS_EINVAL, "run exceeds the collection");
    if (run->mem != COBS_MEM_HOST && run->mem != COBS_MEM_DEVICE)
        return set_error(COBS_EINVAL, "docs.mem must be COBS_MEM_HOST or COBS_MEM_DEVICE");
    if (run->n_docs == 0) return COBS_OK;
    if (!run->str_off || !run->doc_str) return set_error(COBS_EINVAL, "docs offsets are NULL");
    const uint64_t ns = run->doc_str[run->n_docs];
    for (uint32_t d = 0; d < run->n_docs; ++d)
        if (run->doc_str[d + 1] < run->doc_str[d])
            return set_error(COBS_EINVAL, "doc_str must be non-decreasing");
    for (uint64_t s = run->doc_str[0]; s < ns; ++s)
        if (run->str_off[s + 1] < run->str_off[s])
            return set_error(COBS_EINVAL, "str_off must be non-decreasing");
    if (run->str_off[ns] > run->str_off[run->doc_str[0]] && !run->bytes)
        return set_error(COBS_EINVAL, "docs.bytes is NULL");
    return COBS_OK;
}

uint64_t doc_windows(const cobs_docs *run, uint32_t d, uint32_t q)
{
    uint64_t w = 0;
    for (uint64_t s = run->doc_str[d]; s < run->doc_str[d + 1]; ++s) {
        const uint64_t len = run->str_off[s + 1] - run->str_off[s];
        if (len >= q) w += len - q + 1;
    }
    return w;
}

std::vector<Piece> cut_pieces(const cobs_docs *run, uint32_t q)
{
    std::vector<Piece> out;
    uint32_t d0 = 0;
    uint64_t acc = 0;
    for (uint32_t d = 0; d < run->n_docs; ++d) {
        const uint64_t w = doc_windows(run, d, q);
        if (d > d0 && acc + w > kPieceWindows) {
            out.push_back({d0, d});
            d0 = d;
            acc = 0;
        }
        acc += w;
    }
    if (d0 < run->n_docs) out.push_back({d0, run->n_docs});
    return out;
}

// Device bytes and string table of one piece; returns windows in *W.
cobs_status stage_piece(cobs_builder *b, const cobs_docs *run, const Piece &pc, uint64_t *W,
                        const uint8_t **dbytes, uint32_t *n_strs)
{
    const uint32_t q = b->prm.q;
    const uint64_t s0 = run->doc_str[pc.d0], s1 = run->doc_str[pc.d1];
    const uint64_t byte0 = run->str_off[s0], byte1 = run->str_off[s1];
    std::vector<StrDesc> strs;
    strs.reserve(s1 - s0 + 1);
    uint64_t w = 0;
    for (uint32_t d = pc.d0; d < pc.d1; ++d) {
        for (uint64_t s = run->doc_str[d]; s < run->doc_str[d + 1]; ++s) {
            const uint64_t len = run->str_off[s + 1] - run->str_off[s];
            const uint64_t nw = len >= q ? len - q + 1 : 0;
            if (!nw) continue;
            StrDesc sd{};
            sd.byte_off = run->mem == COBS_MEM_HOST ? run->str_off[s] - byte0 : run->str_off[s];
            sd.wbase = w;
            sd.doc = d - pc.d0;
            strs.push_back(sd);
            w += nw;
        }
    }
    StrDesc sentinel{};
    sentinel.wbase = w;
    strs.push_back(sentinel);
    *W = w;
    *n_strs = (uint32_t)strs.size() - 1;
    COBS_HIP(b->strs.ensure(strs.size() * sizeof(StrDesc)));
    COBS_HIP(hipMemcpyAsync(b->strs.p, strs.data(), strs.size() * sizeof(StrDesc),
                            hipMemcpyHostToDevice, b->st));
    if (run->mem == COBS_MEM_HOST) {
        COBS_HIP(b->bytes.ensure(byte1 - byte0 + 64));
        if (byte1 > byte0)
            COBS_HIP(hipMemcpyAsync(b->bytes.p, run->bytes + byte0, byte1 - byte0,
                                    hipMemcpyHostToDevice, b->st));
        *dbytes = b->bytes.as<uint8_t>();
    } else {
        *dbytes = run->bytes;
    }
    return COBS_OK;
}

}  // namespace

extern "C" {

cobs_status cobs_set_allocator(const cobs_allocator *a)
{
    if (a && a->alloc && !a->free) return set_error(COBS_EINVAL, "an allocator needs a free function");
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_alloc = (a && a->alloc) ? *a : cobs_allocator{};
    return COBS_OK;
}

}  // extern "C"

extern "C" {

const char *cobs_last_error(void) { return g_err.c_str(); }

uint64_t cobs_now_ns(void) { return now_ns(); }

cobs_status cobs_builder_create(const cobs_params *params, uint32_t n_docs, void *stream,
                                cobs_builder **out)
{
    if (!out) return set_error(COBS_EINVAL, "out is NULL");
    *out = nullptr;
    cobs_status s = check_params(params);
    if (s != COBS_OK) return s;
    auto *b = new cobs_builder();
    b->prm = *params;
    if (b->prm.kind != COBS_TERMS_DNA) b->prm.canonical = 0;
    b->n_docs = n_docs;
    b->st = (hipStream_t)stream;
    (void)hipGetDevice(&b->device);
    b->n_terms.assign(n_docs, 0);
    b->counted.assign(n_docs, 0);
    b->inserted.assign(n_docs, 0);
    *out = b;
    return COBS_OK;
}

void cobs_builder_free(cobs_builder *b) { delete b; }

cobs_status cobs_builder_count(cobs_builder *b, const cobs_docs *run, uint32_t first)
{
    if (!b) return set_error(COBS_EINVAL, "builder is NULL");
    if (b->state != 0) return set_error(COBS_ESTATE, "count after plan");
    cobs_status s = check_run(b, run, first);
    if (s != COBS_OK) return s;
    const TermSpec ts = term_spec(b->prm);
    for (const Piece &pc : cut_pieces(run, b->prm.q)) {
        uint64_t W;
        const uint8_t *dbytes;
        uint32_t n_strs;
        s = stage_piece(b, run, pc, &W, &dbytes, &n_strs);
        if (s != COBS_OK) return s;
        const uint32_t nd = pc.d1 - pc.d0;
        std::vector<uint64_t> tb(nd);
        std::vector<uint32_t> tl(nd);
        uint64_t slots = 0;
        for (uint32_t i = 0; i < nd; ++i) {
            const uint64_t cap = dedup_table_cap(doc_windows(run, pc.d0 + i, b->prm.q));
            uint32_t lg = 0;
            while ((1ull << lg) < cap) ++lg;
            tb[i] = slots;
            tl[i] = lg;
            slots += cap;
        }
        COBS_HIP(b->tbase.ensure(nd * 8));
        COBS_HIP(b->tlog2.ensure(nd * 4));
        COBS_HIP(b->table.ensure(slots * 8));
        COBS_HIP(b->eflag.ensure(nd * 4));
        COBS_HIP(b->counts.ensure(nd * 8));
        COBS_HIP(hipMemcpyAsync(b->tbase.p, tb.data(), nd * 8, hipMemcpyHostToDevice, b->st));
        COBS_HIP(hipMemcpyAsync(b->tlog2.p, tl.data(), nd * 4, hipMemcpyHostToDevice, b->st));
        COBS_HIP(launch_fill_u64(b->table.as<uint64_t>(), slots, ~0ull, b->st));
        COBS_HIP(hipMemsetAsync(b->eflag.p, 0, nd * 4, b->st));
        COBS_HIP(hipMemsetAsync(b->counts.p, 0, nd * 8, b->st));
        COBS_HIP(launch_count(dbytes, b->strs.as<StrDesc>(), n_strs, W, b->tbase.as<uint64_t>(),
                              b->tlog2.as<uint32_t>(), b->table.as<uint64_t>(),
                              b->eflag.as<uint32_t>(),
                              b->counts.as<unsigned long long>(), ts, b->st));
        std::vector<uint64_t> cnt(nd);
        COBS_HIP(hipMemcpyAsync(cnt.data(), b->counts.p, nd * 8, hipMemcpyDeviceToHost, b->st));
        COBS_HIP(hipStreamSynchronize(b->st));
        for (uint32_t i = 0; i < nd; ++i) {
            b->n_terms[first + pc.d0 + i] = cnt[i];
            b->counted[first + pc.d0 + i] = 1;
        }
    }
    return COBS_OK;
}

}  // extern "C"

namespace cobs {

// The index layout for a given order and block sizes (ix->prm, n_docs,
// n_terms, order set): each block's row count from its largest distinct-term
// count, padded rows, column slices and score-buffer offsets.  Host only.
cobs_status layout_blocks(cobs_index *ix, const std::vector<uint32_t> &block_docs)
{
    ix->seeds = make_seeds(ix->prm.seed);
    ix->blocks.clear();
    ix->slices.clear();
    ix->acc_words = 0;
    uint64_t off = 0;
    uint32_t first = 0;
    for (uint32_t k = 0; k < block_docs.size(); ++k) {
        Block blk{};
        blk.first = first;
        blk.docs = block_docs[k];
        if (blk.docs == 0 || (uint64_t)first + blk.docs > ix->n_docs)
            return set_error(COBS_EINVAL, "block sizes do not cover the documents");
        first += blk.docs;
        for (uint32_t j = 0; j < blk.docs; ++j)
            blk.nmax = std::max(blk.nmax, ix->n_terms[ix->order[blk.first + j]]);
        blk.rows = filter_rows(blk.nmax, ix->prm.num_hashes, ix->prm.fpr);
        if (blk.rows > 0xFFFFFFFFull) return set_error(COBS_EINVAL, "block filter exceeds 2^32-1 rows");
        blk.stride = ((blk.docs + 7) / 8 + 127) / 128 * 128;
        blk.offset = off;
        off += blk.rows * blk.stride;
        off = (off + 255) & ~uint64_t(255);
        ix->blocks.push_back(blk);
        for (uint64_t s0 = 0; s0 < blk.stride; s0 += kSliceBytes) {
            SliceDesc sd{};
            sd.base = blk.offset + s0;
            sd.stride = (uint32_t)blk.stride;
            sd.rows = (uint32_t)blk.rows;
            sd.width = (uint32_t)std::min<uint64_t>(kSliceBytes, blk.stride - s0);
            const uint64_t dfirst = s0 * 8;
            sd.ndocs = (uint32_t)(dfirst < blk.docs ? std::min<uint64_t>(kSliceBytes * 8, blk.docs - dfirst) : 0);
            sd.doc0 = blk.first + (uint32_t)dfirst;
            sd.block = k;
            sd.lanes = (sd.ndocs + 127) / 128;
            sd.acc_off = (uint32_t)ix->acc_words;
            ix->acc_words += 128ull * sd.lanes;
            ix->slices.push_back(sd);
        }
    }
    if (first != ix->n_docs) return set_error(COBS_EINVAL, "block sizes do not cover the documents");
    if (ix->acc_words > 0xFFFFFFFFull) return set_error(COBS_EINVAL, "too many documents for one index");
    ix->total_bytes = off;
    return COBS_OK;
}

// The layout a build gives (ix->prm, n_docs, n_terms set): compact order
// sorted by (distinct terms, input id) (sections 2.2, 2.3) and blocks of B,
// the last one possibly partial; classic: input order, one block.
cobs_status make_layout(cobs_index *ix)
{
    const uint32_t n = ix->n_docs, B = ix->prm.block_docs;
    ix->order.resize(n);
    std::iota(ix->order.begin(), ix->order.end(), 0u);
    if (B) {
        std::stable_sort(ix->order.begin(), ix->order.end(), [&](uint32_t x, uint32_t y) {
            return ix->n_terms[x] < ix->n_terms[y];
        });
    }
    std::vector<uint32_t> sizes;
    for (uint32_t f = 0; f < n; f += B ? B : n) sizes.push_back(B ? std::min(B, n - f) : n);
    return layout_blocks(ix, sizes);
}

// Device copies of the order and the slice table.
cobs_status upload_layout(cobs_index *ix, hipStream_t st)
{
    const uint32_t n = ix->n_docs;
    COBS_HIP(dev_alloc(&ix->d_order, std::max<size_t>(n, 1) * 4));
    if (n) COBS_HIP(hipMemcpyAsync(ix->d_order, ix->order.data(), n * 4, hipMemcpyHostToDevice, st));
    COBS_HIP(dev_alloc(&ix->d_slices, std::max<size_t>(ix->slices.size(), 1) * sizeof(SliceDesc)));
    if (!ix->slices.empty())
        COBS_HIP(hipMemcpyAsync(ix->d_slices, ix->slices.data(), ix->slices.size() * sizeof(SliceDesc),
                                hipMemcpyHostToDevice, st));
    ix->packed = !ix->slices.empty();
    for (const SliceDesc &sd : ix->slices) ix->packed = ix->packed && sd.width <= kPackedSliceBytes;
    return COBS_OK;
}

}  // namespace cobs

extern "C" {

cobs_status cobs_builder_plan(cobs_builder *b)
{
    if (!b) return set_error(COBS_EINVAL, "builder is NULL");
    if (b->state != 0) return set_error(COBS_ESTATE, "plan called twice");
    for (uint32_t d = 0; d < b->n_docs; ++d)
        if (!b->counted[d]) return set_error(COBS_ESTATE, "document " + std::to_string(d) + " not counted");
    auto *ix = new cobs_index();
    ix->prm = b->prm;
    ix->device = b->device;
    ix->n_docs = b->n_docs;
    ix->n_terms = b->n_terms;
    cobs_status s = make_layout(ix);
    if (s != COBS_OK) {
        delete ix;
        return s;
    }
    b->ix = ix;
    const uint64_t off = ix->total_bytes;
    if (off) {
        hipError_t e = dev_alloc(&ix->d_matrix, off);
        if (e != hipSuccess) return hip_error(e, "device memory for the matrix");
        COBS_HIP(hipMemsetAsync(ix->d_matrix, 0, off, b->st));
    }
    s = upload_layout(ix, b->st);
    if (s != COBS_OK) return s;
    const uint32_t n = b->n_docs;
    b->rank.resize(n);
    for (uint32_t p = 0; p < n; ++p) b->rank[ix->order[p]] = p;
    COBS_HIP(hipStreamSynchronize(b->st));
    b->state = 1;
    return COBS_OK;
}

cobs_status cobs_builder_insert(cobs_builder *b, const cobs_docs *run, uint32_t first)
{
    if (!b) return set_error(COBS_EINVAL, "builder is NULL");
    if (b->state != 1) return set_error(COBS_ESTATE, "insert before plan or after finish");
    cobs_status s = check_run(b, run, first);
    if (s != COBS_OK) return s;
    cobs_index *ix = b->ix;
    const TermSpec ts = term_spec(b->prm);
    const uint32_t B = b->prm.block_docs;
    for (const Piece &pc : cut_pieces(run, b->prm.q)) {
        uint64_t W;
        const uint8_t *dbytes;
        uint32_t n_strs;
        s = stage_piece(b, run, pc, &W, &dbytes, &n_strs);
        if (s != COBS_OK) return s;
        const uint32_t nd = pc.d1 - pc.d0;
        std::vector<DocPos> pos(nd);
        for (uint32_t i = 0; i < nd; ++i) {
            const uint32_t id = first + pc.d0 + i;
            const uint32_t p = b->rank[id];
            const uint32_t k = B ? p / B : 0;
            const Block &blk = ix->blocks[k];
            pos[i].block_off = blk.offset;
            pos[i].rows = (uint32_t)blk.rows;
            pos[i].stride = (uint32_t)blk.stride;
            pos[i].col = p - blk.first;
        }
        COBS_HIP(b->pos.ensure(nd * sizeof(DocPos)));
        COBS_HIP(hipMemcpyAsync(b->pos.p, pos.data(), nd * sizeof(DocPos), hipMemcpyHostToDevice, b->st));
        COBS_HIP(launch_insert(dbytes, b->strs.as<StrDesc>(), n_strs, W, b->pos.as<DocPos>(),
                               (uint32_t *)ix->d_matrix, ts, ix->seeds, b->st));
        COBS_HIP(hipStreamSynchronize(b->st));
        for (uint32_t i = 0; i < nd; ++i) b->inserted[first + pc.d0 + i] = 1;
    }
    return COBS_OK;
}

cobs_status cobs_builder_finish(cobs_builder *b, cobs_index **out)
{
    if (!b || !out) return set_error(COBS_EINVAL, "NULL argument");
    if (b->state != 1) return set_error(COBS_ESTATE, "finish before plan");
    for (uint32_t d = 0; d < b->n_docs; ++d)
        if (!b->inserted[d]) return set_error(COBS_ESTATE, "document " + std::to_string(d) + " not inserted");
    COBS_HIP(hipStreamSynchronize(b->st));
    *out = b->ix;
    b->ix = nullptr;
    b->state = 2;
    return COBS_OK;
}

cobs_status cobs_build(const cobs_params *params, const cobs_docs *docs, void *stream,
                       cobs_index **out)
{
    if (!docs || !out) return set_error(COBS_EINVAL, "NULL argument");
    *out = nullptr;
    cobs_builder *b = nullptr;
    cobs_status s = cobs_builder_create(params, docs->n_docs, stream, &b);
    if (s == COBS_OK) s = cobs_builder_count(b, docs, 0);
    if (s == COBS_OK) s = cobs_builder_plan(b);
    if (s == COBS_OK) s = cobs_builder_insert(b, docs, 0);
    if (s == COBS_OK) s = cobs_builder_finish(b, out);
    delete b;
    return s;
}

void cobs_index_free(cobs_index *ix) { delete ix; }

cobs_status cobs_index_info(const cobs_index *ix, cobs_index_info_t *info)
{
    if (!ix || !info) return set_error(COBS_EINVAL, "NULL argument");
    info->n_docs = ix->n_docs;
    info->n_blocks = (uint32_t)ix->blocks.size();
    info->params = ix->prm;
    info->total_bytes = ix->total_bytes;
    info->score_bytes = ix->acc_words * 4;
    info->host_resident = ix->h_matrix ? 1 : 0;
    info->stage_bytes = ix->stage_bytes;
    info->n_groups = (uint32_t)ix->groups.size();
    return COBS_OK;
}

cobs_status cobs_index_block(const cobs_index *ix, uint32_t b, uint32_t *first, uint32_t *docs,
                             uint64_t *rows, uint64_t *stride, uint64_t *offset)
{
    if (!ix) return set_error(COBS_EINVAL, "index is NULL");
    if (b >= ix->blocks.size()) return set_error(COBS_EINVAL, "block out of range");
    const Block &k = ix->blocks[b];
    if (first) *first = k.first;
    if (docs) *docs = k.docs;
    if (rows) *rows = k.rows;
    if (stride) *stride = k.stride;
    if (offset) *offset = k.offset;
    return COBS_OK;
}

cobs_status cobs_index_order(const cobs_index *ix, uint32_t *order, uint64_t *n_terms)
{
    if (!ix) return set_error(COBS_EINVAL, "index is NULL");
    if (order) std::memcpy(order, ix->order.data(), ix->order.size() * 4);
    if (n_terms) std::memcpy(n_terms, ix->n_terms.data(), ix->n_terms.size() * 8);
    return COBS_OK;
}

cobs_status cobs_index_read(const cobs_index *ix, uint64_t offset, uint64_t nbytes, void *dst)
{
    if (!ix || (!dst && nbytes)) return set_error(COBS_EINVAL, "NULL argument");
    if (offset > ix->total_bytes || nbytes > ix->total_bytes - offset)
        return set_error(COBS_EINVAL, "range outside the matrix");
    if (!nbytes) return COBS_OK;
    if (ix->h_matrix)
        std::memcpy(dst, ix->h_matrix + offset, nbytes);
    else
        COBS_HIP(hipMemcpy(dst, ix->d_matrix + offset, nbytes, hipMemcpyDeviceToHost));
    return COBS_OK;
}

}  // extern "C"
