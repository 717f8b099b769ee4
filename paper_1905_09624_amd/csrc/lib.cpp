// COBS library: construction, resident index, query batches, C ABI.
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

void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
}

hipError_t DevBuf::ensure(size_t bytes, bool zero, hipStream_t st)
{
    if (bytes <= cap && p) return hipSuccess;
    release();
    size_t want = bytes < 256 ? 256 : bytes + bytes / 4;
    want = (want + 255) & ~size_t(255);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
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
}

// process-wide gather timing (cobs_profile)
static std::atomic<int> g_prof{0};
static std::mutex g_prof_mu;
static cobs_kernel_timing g_prof_acc{};

static cobs_status check_params(const cobs_params *p)
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

static TermSpec term_spec(const cobs_params &p)
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
        if (d_stage[i]) (void)hipFree(d_stage[i]);
        if (ev_copy[i]) (void)hipEventDestroy(ev_copy[i]);
        if (ev_done[i]) (void)hipEventDestroy(ev_done[i]);
        d_stage[i] = nullptr;
        ev_copy[i] = ev_done[i] = nullptr;
    }
    if (copy_stream) (void)hipStreamDestroy(copy_stream);
    if (d_group_slices) (void)hipFree(d_group_slices);
    if (h_matrix) (void)hipHostFree(h_matrix);
    copy_stream = nullptr;
    d_group_slices = nullptr;
    h_matrix = nullptr;
    groups.clear();
    stage_bytes = 0;
}

cobs_index::~cobs_index()
{
    for (Workspace *w : pool) delete w;
    release_offload();
    if (d_matrix) (void)hipFree(d_matrix);
    if (d_order) (void)hipFree(d_order);
    if (d_slices) (void)hipFree(d_slices);
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

namespace {

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
    COBS_HIP(hipMalloc(&ix->d_order, std::max<size_t>(n, 1) * 4));
    if (n) COBS_HIP(hipMemcpyAsync(ix->d_order, ix->order.data(), n * 4, hipMemcpyHostToDevice, st));
    COBS_HIP(hipMalloc(&ix->d_slices, std::max<size_t>(ix->slices.size(), 1) * sizeof(SliceDesc)));
    if (!ix->slices.empty())
        COBS_HIP(hipMemcpyAsync(ix->d_slices, ix->slices.data(), ix->slices.size() * sizeof(SliceDesc),
                                hipMemcpyHostToDevice, st));
    return COBS_OK;
}

}  // namespace

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
        hipError_t e = hipMalloc(&ix->d_matrix, off);
        if (e != hipSuccess) { ix->d_matrix = nullptr; return hip_error(e, "hipMalloc(matrix)"); }
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

namespace {

// Groups of whole consecutive blocks, each within half the device budget.
cobs_status plan_groups(const cobs_index *ix, uint64_t device_budget_bytes,
                        std::vector<cobs_index::Group> &groups, uint64_t &stage)
{
    const uint64_t half = device_budget_bytes / 2 & ~uint64_t(255);
    groups.clear();
    uint32_t s0 = 0;
    for (size_t b = 0; b < ix->blocks.size(); ++b) {
        const Block &blk = ix->blocks[b];
        const uint64_t end = blk.offset + blk.rows * blk.stride;
        uint32_t ns = 0;
        while (s0 + ns < ix->slices.size() && ix->slices[s0 + ns].block == b) ++ns;
        if (end - blk.offset > half)
            return set_error(COBS_EBUDGET, "half the device budget must hold the largest block (" +
                                                std::to_string(end - blk.offset) + " bytes)");
        if (!groups.empty() && end - groups.back().off <= half) {
            groups.back().bytes = end - groups.back().off;
            groups.back().n_slices += ns;
        } else {
            groups.push_back(cobs_index::Group{s0, ns, blk.offset, end - blk.offset});
        }
        s0 += ns;
    }
    stage = 0;
    for (const auto &gr : groups) stage = std::max(stage, gr.bytes);
    return COBS_OK;
}

// Staging buffers, events, copy stream and rebased slices of a host-resident
// matrix (ix->h_matrix set); on failure the caller releases the offload state.
cobs_status setup_staging(cobs_index *ix, const std::vector<cobs_index::Group> &groups, uint64_t stage)
{
    std::vector<SliceDesc> rebased = ix->slices;
    for (const auto &gr : groups)
        for (uint32_t i = 0; i < gr.n_slices; ++i) rebased[gr.slice0 + i].base -= gr.off;
    for (int i = 0; i < 2; ++i) {
        if (stage) COBS_HIP(hipMalloc(&ix->d_stage[i], stage));
        COBS_HIP(hipEventCreateWithFlags(&ix->ev_copy[i], hipEventDisableTiming));
        COBS_HIP(hipEventCreateWithFlags(&ix->ev_done[i], hipEventDisableTiming));
    }
    COBS_HIP(hipStreamCreateWithFlags(&ix->copy_stream, hipStreamNonBlocking));
    COBS_HIP(hipMalloc(&ix->d_group_slices, std::max<size_t>(rebased.size(), 1) * sizeof(SliceDesc)));
    if (!rebased.empty())
        COBS_HIP(hipMemcpy(ix->d_group_slices, rebased.data(), rebased.size() * sizeof(SliceDesc),
                           hipMemcpyHostToDevice));
    ix->groups = groups;
    ix->stage_bytes = stage;
    return COBS_OK;
}

}  // namespace

cobs_status cobs_index_offload(cobs_index *ix, uint64_t device_budget_bytes)
{
    if (!ix) return set_error(COBS_EINVAL, "index is NULL");
    std::lock_guard<std::mutex> g(ix->stream_mu);
    if (ix->h_matrix) return set_error(COBS_ESTATE, "the matrix is already in host memory");
    (void)hipSetDevice(ix->device);
    std::vector<cobs_index::Group> groups;
    uint64_t stage = 0;
    cobs_status s = plan_groups(ix, device_budget_bytes, groups, stage);
    if (s != COBS_OK) return s;
    hipError_t e = hipHostMalloc((void **)&ix->h_matrix, std::max<uint64_t>(ix->total_bytes, 1));
    if (e != hipSuccess) {
        ix->h_matrix = nullptr;
        return set_error(COBS_ENOMEM, "pinned host memory for the matrix");
    }
    if (ix->total_bytes &&
        (e = hipMemcpy(ix->h_matrix, ix->d_matrix, ix->total_bytes, hipMemcpyDeviceToHost)) != hipSuccess) {
        ix->release_offload();
        return hip_error(e, "hipMemcpy(matrix to host)");
    }
    if ((s = setup_staging(ix, groups, stage)) != COBS_OK) {
        ix->release_offload();
        return s;
    }
    if (ix->d_matrix) (void)hipFree(ix->d_matrix);
    ix->d_matrix = nullptr;
    return COBS_OK;
}

// ---- index files ------------------------------------------------------------------

namespace {

// File layout, little-endian: FileHeader | order u32[n_docs] |
// n_terms u64[n_docs] | FileBlock[n_blocks] | zero padding to a multiple of
// 4096 | the matrix (total_bytes: the blocks one after another, each at its
// offset, as in device memory).  meta_fnv = FNV-1a 64 over the three arrays.
struct FileHeader {
    char magic[8];             // "COBSMTX1"
    uint32_t header_bytes;     // sizeof(FileHeader)
    uint32_t kind, q, canonical, num_hashes, block_docs;
    double fpr;
    uint64_t seed;
    uint32_t n_docs, n_blocks;
    uint64_t total_bytes, matrix_offset, meta_fnv;
};

struct FileBlock {
    uint32_t first, docs;
    uint64_t rows, stride, offset;
};

constexpr char kFileMagic[8] = {'C', 'O', 'B', 'S', 'M', 'T', 'X', '1'};
constexpr uint64_t kFileChunk = 64ull << 20;

uint64_t fnv1a(uint64_t h, const void *p, size_t n)
{
    const uint8_t *b = static_cast<const uint8_t *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001B3ull;
    return h;
}

struct File {
    FILE *f = nullptr;
    ~File() { if (f) std::fclose(f); }
};

}  // namespace

cobs_status cobs_index_save(const cobs_index *ix, const char *path)
{
    if (!ix || !path) return set_error(COBS_EINVAL, "NULL argument");
    std::vector<FileBlock> fb;
    for (const Block &b : ix->blocks) fb.push_back(FileBlock{b.first, b.docs, b.rows, b.stride, b.offset});
    FileHeader h{};
    std::memcpy(h.magic, kFileMagic, 8);
    h.header_bytes = sizeof(FileHeader);
    h.kind = ix->prm.kind;
    h.q = ix->prm.q;
    h.canonical = ix->prm.canonical;
    h.num_hashes = ix->prm.num_hashes;
    h.block_docs = ix->prm.block_docs;
    h.fpr = ix->prm.fpr;
    h.seed = ix->prm.seed;
    h.n_docs = ix->n_docs;
    h.n_blocks = (uint32_t)fb.size();
    h.total_bytes = ix->total_bytes;
    const uint64_t meta = sizeof(FileHeader) + (uint64_t)ix->n_docs * 12 + fb.size() * sizeof(FileBlock);
    h.matrix_offset = (meta + 4095) & ~uint64_t(4095);
    uint64_t fnv = 0xCBF29CE484222325ull;
    fnv = fnv1a(fnv, ix->order.data(), ix->order.size() * 4);
    fnv = fnv1a(fnv, ix->n_terms.data(), ix->n_terms.size() * 8);
    fnv = fnv1a(fnv, fb.data(), fb.size() * sizeof(FileBlock));
    h.meta_fnv = fnv;
    File out;
    if (!(out.f = std::fopen(path, "wb"))) return set_error(COBS_EINVAL, std::string("cannot create ") + path);
    std::vector<uint8_t> pad(h.matrix_offset - meta, 0);
    bool ok = std::fwrite(&h, sizeof h, 1, out.f) == 1 &&
              std::fwrite(ix->order.data(), 4, ix->n_docs, out.f) == ix->n_docs &&
              std::fwrite(ix->n_terms.data(), 8, ix->n_docs, out.f) == ix->n_docs &&
              std::fwrite(fb.data(), sizeof(FileBlock), fb.size(), out.f) == fb.size() &&
              std::fwrite(pad.data(), 1, pad.size(), out.f) == pad.size();
    if (ok && ix->h_matrix) {
        ok = std::fwrite(ix->h_matrix, 1, ix->total_bytes, out.f) == ix->total_bytes;
    } else if (ok && ix->total_bytes) {
        (void)hipSetDevice(ix->device);
        HostBuf stage;
        COBS_HIP(stage.ensure(std::min(kFileChunk, ix->total_bytes)));
        for (uint64_t o = 0; ok && o < ix->total_bytes; o += kFileChunk) {
            const uint64_t nb = std::min(kFileChunk, ix->total_bytes - o);
            COBS_HIP(hipMemcpy(stage.p, ix->d_matrix + o, nb, hipMemcpyDeviceToHost));
            ok = std::fwrite(stage.p, 1, nb, out.f) == nb;
        }
    }
    if (!ok || std::fflush(out.f) != 0) return set_error(COBS_EINVAL, std::string("write failed: ") + path);
    return COBS_OK;
}

cobs_status cobs_index_load(const char *path, int device, uint64_t device_budget_bytes,
                            cobs_index **out)
{
    if (!path || !out) return set_error(COBS_EINVAL, "NULL argument");
    *out = nullptr;
    File in;
    if (!(in.f = std::fopen(path, "rb"))) return set_error(COBS_EINVAL, std::string("cannot open ") + path);
    auto bad = [&](const char *why) { return set_error(COBS_EINVAL, std::string(path) + ": " + why); };
    FileHeader h{};
    if (std::fread(&h, sizeof h, 1, in.f) != 1) return bad("truncated header");
    if (std::memcmp(h.magic, kFileMagic, 8) != 0 || h.header_bytes != sizeof(FileHeader))
        return bad("not an index file of this format");
    cobs_params prm{};
    prm.kind = h.kind;
    prm.q = h.q;
    prm.canonical = h.canonical;
    prm.num_hashes = h.num_hashes;
    prm.fpr = h.fpr;
    prm.block_docs = h.block_docs;
    prm.seed = h.seed;
    cobs_status s = check_params(&prm);
    if (s != COBS_OK) return s;
    std::unique_ptr<cobs_index> ix(new cobs_index());
    ix->prm = prm;
    ix->device = device;
    ix->n_docs = h.n_docs;
    std::vector<uint32_t> order(h.n_docs);
    ix->n_terms.resize(h.n_docs);
    std::vector<FileBlock> fb(h.n_blocks);
    if (std::fread(order.data(), 4, h.n_docs, in.f) != h.n_docs ||
        std::fread(ix->n_terms.data(), 8, h.n_docs, in.f) != h.n_docs ||
        std::fread(fb.data(), sizeof(FileBlock), h.n_blocks, in.f) != h.n_blocks)
        return bad("truncated metadata");
    uint64_t fnv = 0xCBF29CE484222325ull;
    fnv = fnv1a(fnv, order.data(), order.size() * 4);
    fnv = fnv1a(fnv, ix->n_terms.data(), ix->n_terms.size() * 8);
    fnv = fnv1a(fnv, fb.data(), fb.size() * sizeof(FileBlock));
    if (fnv != h.meta_fnv) return bad("metadata checksum mismatch");
    // the order must be a permutation; the block table must follow from the
    // counts and the block sizes (a merged compact index need not be sorted
    // across its parts, section 2.3)
    {
        std::vector<uint8_t> seen(h.n_docs, 0);
        for (uint32_t d : order) {
            if (d >= h.n_docs || seen[d]) return bad("order is not a permutation");
            seen[d] = 1;
        }
    }
    ix->order = order;
    std::vector<uint32_t> sizes;
    for (const FileBlock &b : fb) sizes.push_back(b.docs);
    if ((s = layout_blocks(ix.get(), sizes)) != COBS_OK) return bad("invalid block table");
    if (ix->blocks.size() != fb.size() || ix->total_bytes != h.total_bytes)
        return bad("layout does not follow from the stored counts");
    for (size_t b = 0; b < fb.size(); ++b) {
        const Block &k = ix->blocks[b];
        if (k.first != fb[b].first || k.docs != fb[b].docs || k.rows != fb[b].rows ||
            k.stride != fb[b].stride || k.offset != fb[b].offset)
            return bad("block table does not follow from the stored counts");
    }
    if (std::fseek(in.f, (long)h.matrix_offset, SEEK_SET) != 0) return bad("truncated");
    COBS_HIP(hipSetDevice(device));
    hipStream_t st = nullptr;
    if ((s = upload_layout(ix.get(), st)) != COBS_OK) return s;
    const uint64_t T = ix->total_bytes;
    if (device_budget_bytes) {
        std::vector<cobs_index::Group> groups;
        uint64_t stage = 0;
        if ((s = plan_groups(ix.get(), device_budget_bytes, groups, stage)) != COBS_OK) return s;
        if (hipHostMalloc((void **)&ix->h_matrix, std::max<uint64_t>(T, 1)) != hipSuccess) {
            ix->h_matrix = nullptr;
            return set_error(COBS_ENOMEM, "pinned host memory for the matrix");
        }
        if (T && std::fread(ix->h_matrix, 1, T, in.f) != T) return bad("truncated matrix");
        if ((s = setup_staging(ix.get(), groups, stage)) != COBS_OK) return s;
    } else {
        if (T) {
            hipError_t e = hipMalloc(&ix->d_matrix, T);
            if (e != hipSuccess) {
                ix->d_matrix = nullptr;
                return set_error(COBS_ENOMEM, "device memory for the matrix");
            }
            HostBuf stage;
            COBS_HIP(stage.ensure(std::min(kFileChunk, T)));
            for (uint64_t o = 0; o < T; o += kFileChunk) {
                const uint64_t nb = std::min(kFileChunk, T - o);
                if (std::fread(stage.p, 1, nb, in.f) != nb) return bad("truncated matrix");
                COBS_HIP(hipMemcpy(ix->d_matrix + o, stage.p, nb, hipMemcpyHostToDevice));
            }
        }
    }
    COBS_HIP(hipDeviceSynchronize());
    *out = ix.release();
    return COBS_OK;
}

cobs_status cobs_index_merge(const cobs_index *a, const cobs_index *b, cobs_index **out)
{
    if (!a || !b || !out) return set_error(COBS_EINVAL, "NULL argument");
    *out = nullptr;
    const cobs_params &p = a->prm, &q = b->prm;
    if (p.kind != q.kind || p.q != q.q || p.canonical != q.canonical || p.num_hashes != q.num_hashes ||
        p.fpr != q.fpr || p.block_docs != q.block_docs || p.seed != q.seed)
        return set_error(COBS_EINVAL, "indexes with different parameters");
    if (a->device != b->device) return set_error(COBS_EINVAL, "indexes on different devices");
    if (a->h_matrix || b->h_matrix) return set_error(COBS_ESTATE, "merge needs both matrices in device memory");
    if ((uint64_t)a->n_docs + b->n_docs > 0xFFFFFFFFull) return set_error(COBS_EINVAL, "too many documents");
    const bool classic = p.block_docs == 0;
    if (classic && a->n_docs && b->n_docs && a->blocks[0].rows != b->blocks[0].rows)
        return set_error(COBS_EINVAL, "classic indexes merge only with equal row counts (" +
                                          std::to_string(a->blocks[0].rows) + " and " +
                                          std::to_string(b->blocks[0].rows) + ")");
    COBS_HIP(hipSetDevice(a->device));
    std::unique_ptr<cobs_index> ix(new cobs_index());
    ix->prm = p;
    ix->device = a->device;
    const uint32_t na = a->n_docs;
    ix->n_docs = na + b->n_docs;
    ix->n_terms = a->n_terms;
    ix->n_terms.insert(ix->n_terms.end(), b->n_terms.begin(), b->n_terms.end());
    ix->order = a->order;
    for (uint32_t d : b->order) ix->order.push_back(d + na);
    std::vector<uint32_t> sizes;
    if (classic) {
        if (ix->n_docs) sizes.push_back(ix->n_docs);
    } else {
        for (const Block &k : a->blocks) sizes.push_back(k.docs);
        for (const Block &k : b->blocks) sizes.push_back(k.docs);
    }
    cobs_status s = layout_blocks(ix.get(), sizes);
    if (s != COBS_OK) return s;
    hipStream_t st = nullptr;
    if (ix->total_bytes) {
        hipError_t e = hipMalloc(&ix->d_matrix, ix->total_bytes);
        if (e != hipSuccess) {
            ix->d_matrix = nullptr;
            return set_error(COBS_ENOMEM, "device memory for the matrix");
        }
    }
    if (classic && ix->n_docs) {
        const Block &o = ix->blocks[0];
        const cobs_index *x = na ? a : b;   // a side with documents gives the row count
        if (o.rows != x->blocks[0].rows) return set_error(COBS_EINVAL, "row counts disagree");
        if (na && b->n_docs) {
            COBS_HIP(launch_concat_rows(a->d_matrix, a->blocks[0].stride, na, b->d_matrix,
                                        b->blocks[0].stride, ix->d_matrix, o.stride, o.rows, st));
        } else {
            COBS_HIP(hipMemcpyAsync(ix->d_matrix, x->d_matrix, x->total_bytes, hipMemcpyDeviceToDevice, st));
        }
    } else if (!classic) {
        size_t k = 0;
        for (const cobs_index *x : {a, b}) {
            for (const Block &src : x->blocks) {
                const Block &dst = ix->blocks[k++];
                if (dst.rows != src.rows || dst.stride != src.stride)
                    return set_error(COBS_EINVAL, "block layout disagrees");
                COBS_HIP(hipMemcpyAsync(ix->d_matrix + dst.offset, x->d_matrix + src.offset,
                                        src.rows * src.stride, hipMemcpyDeviceToDevice, st));
            }
        }
    }
    if ((s = upload_layout(ix.get(), st)) != COBS_OK) return s;
    COBS_HIP(hipStreamSynchronize(st));
    *out = ix.release();
    return COBS_OK;
}

cobs_status cobs_index_onload(cobs_index *ix)
{
    if (!ix) return set_error(COBS_EINVAL, "index is NULL");
    std::lock_guard<std::mutex> g(ix->stream_mu);
    if (!ix->h_matrix) return set_error(COBS_ESTATE, "the matrix is already in device memory");
    (void)hipSetDevice(ix->device);
    uint8_t *d = nullptr;
    hipError_t e = hipMalloc(&d, std::max<uint64_t>(ix->total_bytes, 1));
    if (e != hipSuccess) return set_error(COBS_ENOMEM, "device memory for the matrix");
    if (ix->total_bytes && (e = hipMemcpy(d, ix->h_matrix, ix->total_bytes, hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(d);
        return hip_error(e, "hipMemcpy(matrix to device)");
    }
    ix->d_matrix = d;
    ix->release_offload();
    return COBS_OK;
}

}  // extern "C"

// ---- query batches -------------------------------------------------------------------

namespace cobs {

Workspace *acquire_workspace(cobs_index *ix)
{
    std::lock_guard<std::mutex> g(ix->pool_mu);
    if (!ix->pool.empty()) {
        Workspace *w = ix->pool.back();
        ix->pool.pop_back();
        return w;
    }
    return new Workspace();
}

void release_workspace(cobs_index *ix, Workspace *ws)
{
    std::lock_guard<std::mutex> g(ix->pool_mu);
    ix->pool.push_back(ws);
}

namespace {

struct Scalars {
    uint64_t total_items;
    unsigned long long work_counter;
    unsigned long long cand_counter;
    uint32_t flags;
    uint32_t pad;
};

// qstart, wbase, tbase (u64); slot, lds_q + g_q (n entries together), gprefix (u32)
size_t batch_meta_bytes(uint32_t n)
{
    return ((size_t)n * 8 + (size_t)(n + 1) * 8 + (size_t)n * 8 + (size_t)n * 4 + (size_t)n * 4 +
            (size_t)(n + 1) * 4 + 15) & ~size_t(15);
}

// Terms per work item: enough items to keep every resident wavefront busy
// about twice over (items start largest first, so the last ones are small),
// never more than cap (fewer, longer items; fewer merges) nor fewer than 32
// terms.
uint32_t auto_chunk(uint64_t W, uint32_t n_slices, int grid, uint32_t cap)
{
    const uint64_t waves = (uint64_t)grid * 4;
    uint64_t c = (W * n_slices + 2 * waves - 1) / (2 * waves);
    if (c > cap) c = cap;
    if (c < 32) c = 32;
    return (uint32_t)c;
}

}  // namespace

// The gather of an offloaded index: group by group, the copy of group g + 2
// (on the index's copy stream) overlaps the gathers of groups g and g + 1 (on
// st), through two staging buffers.  The caller holds ix->stream_mu.
static cobs_status gather_streamed(cobs_index *ix, Workspace &ws, GatherArgs ga, int planes, int unroll,
                                   int grid, hipStream_t st)
{
    const size_t G = ix->groups.size();
    COBS_HIP(ws.counters.ensure(G * 8));
    unsigned long long *counters = ws.counters.as<unsigned long long>();
    COBS_HIP(launch_fill_u64((uint64_t *)counters, G, 0, st));
    // the copies start after everything before them on st (earlier batches
    // read the staging buffers)
    COBS_HIP(hipEventRecord(ix->ev_done[0], st));
    COBS_HIP(hipEventRecord(ix->ev_done[1], st));
    auto copy = [&](size_t g) -> cobs_status {
        const cobs_index::Group &gr = ix->groups[g];
        COBS_HIP(hipStreamWaitEvent(ix->copy_stream, ix->ev_done[g % 2], 0));
        COBS_HIP(hipMemcpyAsync(ix->d_stage[g % 2], ix->h_matrix + gr.off, gr.bytes,
                                hipMemcpyHostToDevice, ix->copy_stream));
        COBS_HIP(hipEventRecord(ix->ev_copy[g % 2], ix->copy_stream));
        return COBS_OK;
    };
    for (size_t g = 0; g < std::min<size_t>(G, 2); ++g) {
        cobs_status c = copy(g);
        if (c != COBS_OK) return c;
    }
    for (size_t g = 0; g < G; ++g) {
        const cobs_index::Group &gr = ix->groups[g];
        COBS_HIP(hipStreamWaitEvent(st, ix->ev_copy[g % 2], 0));
        GatherArgs a = ga;
        a.matrix = ix->d_stage[g % 2];
        a.slices = ix->d_group_slices + gr.slice0;
        a.n_slices = gr.n_slices;
        a.work_counter = counters + g;
        COBS_HIP(launch_gather(a, planes, unroll, grid, st));
        COBS_HIP(hipEventRecord(ix->ev_done[g % 2], st));
        if (g + 2 < G) {
            cobs_status c = copy(g + 2);
            if (c != COBS_OK) return c;
        }
    }
    return COBS_OK;
}

cobs_status run_batch(cobs_index *ix, Workspace &ws, const BatchSpec &b, hipStream_t st,
                      BatchOut &out)
{
    std::unique_lock<std::mutex> streaming(ix->stream_mu, std::defer_lock);
    if (ix->h_matrix) streaming.lock();   // one streamed batch at a time
    const uint32_t n = b.n;
    out.num_terms.assign(n, 0);
    out.n.assign(n, 0);
    out.start.assign(n + 1, 0);
    if (n == 0) return COBS_OK;
    if (!b.q_off) return set_error(COBS_EINVAL, "q_off is NULL");
    if (b.k_den == 0) return set_error(COBS_EINVAL, "k_den must be > 0");
    if (b.score_bits != 16 && b.score_bits != 32)
        return set_error(COBS_EINVAL, "score_bits must be 16 or 32");
    if (b.mem != COBS_MEM_HOST && b.mem != COBS_MEM_DEVICE)
        return set_error(COBS_EINVAL, "mem must be COBS_MEM_HOST or COBS_MEM_DEVICE");
    const uint32_t q = ix->prm.q, h = ix->prm.num_hashes;
    const uint32_t n_slices = (uint32_t)ix->slices.size();
    const uint64_t byte0 = b.q_off[0];
    const uint64_t nbytes = b.q_off[n] - b.q_off[0];
    if (nbytes && !b.bytes) return set_error(COBS_EINVAL, "bytes is NULL");

    // host plan: windows, dedup tables, launch shape, score-buffer slots
    std::vector<uint64_t> hv(2 * (size_t)n + 1);
    uint64_t *qstart = hv.data(), *wbase = hv.data() + n;
    uint64_t W = 0, maxw = 0, tslots = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (b.q_off[i + 1] < b.q_off[i]) return set_error(COBS_EINVAL, "q_off must be non-decreasing");
        const uint64_t len = b.q_off[i + 1] - b.q_off[i];
        const uint64_t nw = len >= q ? len - q + 1 : 0;
        qstart[i] = b.q_off[i] - byte0;
        wbase[i] = W;
        W += nw;
        maxw = std::max(maxw, nw);
    }
    wbase[n] = W;
    // dedup work lists: queries with an LDS set; queries with a global table
    // and the first workgroup of each
    std::vector<uint64_t> tb(n, 0);
    std::vector<uint32_t> lds_q, lds_large, g_q, gprefix;
    uint64_t groups = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t nw = wbase[i + 1] - wbase[i];
        const uint64_t slots = dedup_table_slots(nw);
        tb[i] = tslots;
        tslots += slots;
        if (slots) {
            g_q.push_back(i);
            gprefix.push_back((uint32_t)groups);
            groups += dedup_groups(nw);
        } else if (dedup_small_table(nw)) {
            lds_q.push_back(i);
        } else {
            lds_large.push_back(i);
        }
    }
    const uint32_t n_small = (uint32_t)lds_q.size();
    lds_q.insert(lds_q.end(), lds_large.begin(), lds_large.end());
    if (groups > 0x7FFFFFFFull) return set_error(COBS_EINVAL, "query batch too large");
    gprefix.push_back((uint32_t)groups);
    const int planes = gather_planes_for(maxw);
    int unroll = b.unroll ? (int)b.unroll : (ix->tuned_unroll ? ix->tuned_unroll : gather_default_unroll((int)h));
    if (!gather_unroll_valid(unroll, (int)h)) unroll = gather_default_unroll((int)h);
    int grid = gather_grid(planes, unroll, (int)h);
    const uint32_t cap = b.chunk_cap ? b.chunk_cap : (ix->tuned_chunk ? ix->tuned_chunk : kDefaultChunkCap);
    const uint32_t C = b.chunk ? b.chunk : auto_chunk(W, n_slices, grid, cap);
    uint64_t pslots = 0, items = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t nw = wbase[i + 1] - wbase[i];
        if (nw > C) pslots += 1;   // may be split: one score buffer
        items += (nw + C - 1) / C;
    }
    // no more wavefronts than work items (4 per workgroup)
    items *= n_slices;
    if ((uint64_t)grid * 4 > items) grid = (int)std::max<uint64_t>(1, (items + 3) / 4);
    const TermSpec ts = term_spec(ix->prm);

    // uploads
    // staging: qstart | wbase | tbase | slot | lds_q | g_q | gprefix | query bytes (host mode)
    const size_t o_wb = (size_t)n * 8, o_tb = o_wb + (size_t)(n + 1) * 8, o_sl = o_tb + (size_t)n * 8;
    const size_t o_lq = o_sl + (size_t)n * 4, o_gq = o_lq + lds_q.size() * 4;
    const size_t o_gp = o_gq + g_q.size() * 4;
    const size_t meta = batch_meta_bytes(n);
    COBS_HIP(ws.h_stage.ensure(meta + (b.mem == COBS_MEM_HOST ? nbytes : 0)));
    uint8_t *stg = ws.h_stage.as<uint8_t>();
    std::memcpy(stg, qstart, (size_t)n * 8);
    std::memcpy(stg + o_wb, wbase, (size_t)(n + 1) * 8);
    std::memcpy(stg + o_tb, tb.data(), (size_t)n * 8);
    if (b.slots) std::memcpy(stg + o_sl, b.slots, (size_t)n * 4);
    std::memcpy(stg + o_lq, lds_q.data(), lds_q.size() * 4);
    std::memcpy(stg + o_gq, g_q.data(), g_q.size() * 4);
    std::memcpy(stg + o_gp, gprefix.data(), gprefix.size() * 4);
    COBS_HIP(ws.meta.ensure(meta));
    COBS_HIP(hipMemcpyAsync(ws.meta.p, stg, meta, hipMemcpyHostToDevice, st));
    const uint64_t *d_qstart = ws.meta.as<uint64_t>();
    const uint64_t *d_wbase = (const uint64_t *)(ws.meta.as<uint8_t>() + o_wb);
    const uint64_t *d_tbase = (const uint64_t *)(ws.meta.as<uint8_t>() + o_tb);
    const uint32_t *d_slot = b.slots ? (const uint32_t *)(ws.meta.as<uint8_t>() + o_sl) : nullptr;
    const uint32_t *d_lds_q = (const uint32_t *)(ws.meta.as<uint8_t>() + o_lq);
    const uint32_t *d_g_q = (const uint32_t *)(ws.meta.as<uint8_t>() + o_gq);
    const uint32_t *d_gprefix = (const uint32_t *)(ws.meta.as<uint8_t>() + o_gp);
    // the query bytes in the workspace (256-byte aligned, 64 bytes of slack:
    // the extract kernel reads whole aligned dwords around each window)
    COBS_HIP(ws.bytes.ensure(nbytes + 64));
    if (nbytes && b.mem == COBS_MEM_HOST) {
        std::memcpy(stg + meta, b.bytes + byte0, nbytes);
        COBS_HIP(hipMemcpyAsync(ws.bytes.p, stg + meta, nbytes, hipMemcpyHostToDevice, st));
    } else if (nbytes) {
        COBS_HIP(hipMemcpyAsync(ws.bytes.p, b.bytes + byte0, nbytes, hipMemcpyDeviceToDevice, st));
    }
    const uint8_t *dbytes = ws.bytes.as<uint8_t>();

    // a1-a3
    COBS_HIP(ws.terms.ensure(std::max<uint64_t>(W, 1) * 8));
    COBS_HIP(ws.uterms.ensure(std::max<uint64_t>(W, 1) * 8));
    COBS_HIP(ws.hashes.ensure(std::max<uint64_t>(W, 1) * 8 * h));
    // result head, copied back in one piece: Scalars | nterms[n] | out_n[n] | out_start[n + 1]
    const size_t head_bytes = sizeof(Scalars) + (size_t)n * 8 + (size_t)(n + 1) * 4;
    COBS_HIP(ws.head.ensure(head_bytes));
    Scalars *dsc = ws.head.as<Scalars>();
    uint32_t *d_nterms = (uint32_t *)(ws.head.as<uint8_t>() + sizeof(Scalars));
    uint32_t *d_out_n = d_nterms + n;
    uint32_t *d_out_start = d_out_n + n;
    COBS_HIP(ws.table.ensure(std::max<uint64_t>(tslots, 1) * 8));
    COBS_HIP(launch_extract(dbytes, d_qstart, d_wbase, n, W, ts, ws.terms.as<uint64_t>(), d_nterms,
                            st));
    COBS_HIP(launch_dedup(ws.terms.as<uint64_t>(), d_wbase, d_tbase, d_lds_q, n_small,
                          (uint32_t)lds_large.size(), d_g_q, d_gprefix, (uint32_t)g_q.size(),
                          (uint32_t)groups, ws.table.as<uint64_t>(), tslots,
                          ws.uterms.as<uint64_t>(), ws.hashes.as<uint64_t>(), d_nterms, ts,
                          ix->seeds, st));
    if (b.terms_out) {
        std::vector<uint32_t> nt(n);
        COBS_HIP(hipMemcpyAsync(nt.data(), d_nterms, (size_t)n * 4, hipMemcpyDeviceToHost, st));
        if (W) COBS_HIP(hipMemcpyAsync(b.terms_out, ws.uterms.p, W * 8, hipMemcpyDeviceToHost, st));
        COBS_HIP(hipStreamSynchronize(st));
        out.num_terms = nt;
        return COBS_OK;
    }

    // a4-a8
    const uint64_t tslots_need = (uint64_t)n * n_slices;
    if (ws.tickets_slots < tslots_need || !ws.tickets.p) {
        COBS_HIP(ws.tickets.ensure(std::max<uint64_t>(tslots_need, 1) * 4, true, st));
        ws.tickets_slots = ws.tickets.cap / 4;
    }
    COBS_HIP(ws.qinfo.ensure((size_t)n * sizeof(QInfo)));
    COBS_HIP(ws.chunk_prefix.ensure((size_t)(n + 1) * 4));
    COBS_HIP(ws.qorder.ensure((size_t)n * 4));
    // score buffers of split queries: zero on allocation, left zero by every
    // complete gather launch
    uint32_t *accum = b.accum;
    if (!accum) {
        const uint64_t accum_words = pslots * ix->acc_words;
        if (ws.accum_words < accum_words || !ws.accum.p) {
            COBS_HIP(ws.accum.ensure(std::max<uint64_t>(accum_words, 64) * 4, true, st));
            ws.accum_words = ws.accum.cap / 4;
        }
        accum = ws.accum.as<uint32_t>();
    }
    COBS_HIP(ws.qcount.ensure((size_t)n * 4));
    const uint64_t ell_limit = b.score_bits == 16 ? 0xFFFFull : 0xFFFFFFFFull;
    const bool full = b.full_scores != nullptr;
    if (ws.cand_cap == 0) ws.cand_cap = std::max<uint64_t>(1 << 20, (uint64_t)n * 64);

    for (int attempt = 0;; ++attempt) {
        COBS_HIP(ws.cand_key.ensure(ws.cand_cap * 8));
        COBS_HIP(ws.cand_q.ensure(ws.cand_cap * 4));
        COBS_HIP(launch_plan(d_nterms, d_wbase, d_slot, n, C, n_slices,
                             b.k_num, b.k_den, ell_limit, ws.qinfo.as<QInfo>(),
                             ws.qorder.as<uint32_t>(), ws.chunk_prefix.as<uint32_t>(),
                             &dsc->total_items, &dsc->work_counter, &dsc->cand_counter,
                             ws.qcount.as<uint32_t>(), &dsc->flags, st));
        if (full) {
            COBS_HIP(ws.full.ensure(std::max<uint64_t>((uint64_t)n * ix->n_docs, 1) * 4));
            COBS_HIP(hipMemsetAsync(ws.full.p, 0, (uint64_t)n * ix->n_docs * 4, st));
        }
        GatherArgs ga{};
        ga.matrix = ix->d_matrix;
        ga.slices = ix->d_slices;
        ga.order = ix->d_order;
        ga.hashes = ws.hashes.as<uint64_t>();
        ga.qinfo = ws.qinfo.as<QInfo>();
        ga.qorder = ws.qorder.as<uint32_t>();
        ga.chunk_prefix = ws.chunk_prefix.as<uint32_t>();
        ga.work_counter = &dsc->work_counter;
        ga.tickets = ws.tickets.as<uint32_t>();
        ga.accum = accum;
        ga.acc_words = ix->acc_words;
        ga.cand_counter = &dsc->cand_counter;
        ga.cand_key = ws.cand_key.as<uint64_t>();
        ga.cand_q = ws.cand_q.as<uint32_t>();
        ga.qcount = ws.qcount.as<uint32_t>();
        ga.full_scores = full ? ws.full.as<uint32_t>() : nullptr;
        ga.cand_cap = ws.cand_cap;
        ga.n_queries = n;
        ga.n_slices = n_slices;
        ga.h = h;
        ga.chunk = C;
        ga.topk = b.topk;
        ga.n_docs = ix->n_docs;
        const bool prof = g_prof.load() != 0;
        const bool timed = prof || b.time_gather;
        if (timed) {
            for (hipEvent_t &e : ws.ev)
                if (!e) COBS_HIP(hipEventCreate(&e));
            COBS_HIP(hipEventRecord(ws.ev[0], st));
        }
        if (n_slices && !ix->h_matrix) COBS_HIP(launch_gather(ga, planes, unroll, grid, st));
        if (n_slices && ix->h_matrix) {
            cobs_status gs = gather_streamed(ix, ws, ga, planes, unroll, grid, st);
            if (gs != COBS_OK) return gs;
        }
        if (timed) COBS_HIP(hipEventRecord(ws.ev[1], st));
        auto account = [&](const uint32_t *nt) -> cobs_status {
            if (!timed) return COBS_OK;
            float ms = 0.f;
            COBS_HIP(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[1]));
            out.gather_ms = ms;
            if (!prof) return COBS_OK;
            uint64_t terms = 0, per_term = 0;
            for (uint32_t i = 0; i < n; ++i) terms += nt[i];
            for (const SliceDesc &sd : ix->slices) per_term += sd.width;
            std::lock_guard<std::mutex> g(g_prof_mu);
            g_prof_acc.launches += 1;
            g_prof_acc.total_ms += ms;
            g_prof_acc.last_ms = ms;
            g_prof_acc.terms += terms;
            g_prof_acc.row_bytes += terms * h * per_term;
            return COBS_OK;
        };
        if (full) {
            const size_t nb = sizeof(Scalars) + (size_t)n * 4;
            COBS_HIP(ws.h_small.ensure(nb));
            COBS_HIP(hipMemcpyAsync(ws.h_small.p, ws.head.p, nb, hipMemcpyDeviceToHost, st));
            if (ix->n_docs)
                COBS_HIP(hipMemcpyAsync(b.full_scores, ws.full.p, (uint64_t)n * ix->n_docs * 4,
                                        hipMemcpyDeviceToHost, st));
            COBS_HIP(hipStreamSynchronize(st));
            Scalars hs;
            std::memcpy(&hs, ws.h_small.p, sizeof(Scalars));
            std::memcpy(out.num_terms.data(), ws.h_small.as<uint8_t>() + sizeof(Scalars), (size_t)n * 4);
            if (hs.flags & 1u) return set_error(COBS_EOVERFLOW, "a query exceeds the score width");
            return account(out.num_terms.data());
        }
        COBS_HIP(ws.gstart.ensure((size_t)(n + 1) * 4));
        COBS_HIP(ws.gcursor.ensure((size_t)n * 4));
        COBS_HIP(ws.seg_a.ensure(ws.cand_cap * 8));
        COBS_HIP(ws.seg_b.ensure(ws.cand_cap * 8));
        COBS_HIP(ws.out_id.ensure(ws.cand_cap * 4));
        COBS_HIP(ws.out_score.ensure(ws.cand_cap * 4));
        COBS_HIP(launch_group_sort(ws.cand_key.as<uint64_t>(), ws.cand_q.as<uint32_t>(),
                                   &dsc->cand_counter, ws.cand_cap, n, b.topk,
                                   ws.qcount.as<uint32_t>(), ws.gstart.as<uint32_t>(),
                                   ws.gcursor.as<uint32_t>(), ws.seg_a.as<uint64_t>(),
                                   ws.seg_b.as<uint64_t>(), d_out_start, d_out_n,
                                   ws.out_id.as<uint32_t>(), ws.out_score.as<uint32_t>(), st));
        COBS_HIP(ws.h_small.ensure(head_bytes));
        uint8_t *hs = ws.h_small.as<uint8_t>();
        COBS_HIP(hipMemcpyAsync(hs, ws.head.p, head_bytes, hipMemcpyDeviceToHost, st));
        COBS_HIP(hipStreamSynchronize(st));
        Scalars sc;
        std::memcpy(&sc, hs, sizeof(Scalars));
        {
            cobs_status a = account((const uint32_t *)(hs + sizeof(Scalars)));
            if (a != COBS_OK) return a;
        }
        if (sc.flags & 1u) return set_error(COBS_EOVERFLOW, "a query exceeds the score width");
        if (sc.cand_counter > ws.cand_cap) {
            if (attempt >= 2) return set_error(COBS_EDEVICE, "candidate buffer kept overflowing");
            ws.cand_cap = sc.cand_counter + sc.cand_counter / 4 + 1024;
            continue;
        }
        std::memcpy(out.num_terms.data(), hs + sizeof(Scalars), (size_t)n * 4);
        std::memcpy(out.n.data(), hs + sizeof(Scalars) + (size_t)n * 4, (size_t)n * 4);
        std::memcpy(out.start.data(), hs + sizeof(Scalars) + (size_t)n * 8, (size_t)(n + 1) * 4);
        const uint64_t total = out.start[n];
        COBS_HIP(ws.h_out.ensure(std::max<uint64_t>(total, 1) * 8));
        uint32_t *ho = ws.h_out.as<uint32_t>();
        if (total) {
            COBS_HIP(hipMemcpyAsync(ho, ws.out_id.p, total * 4, hipMemcpyDeviceToHost, st));
            COBS_HIP(hipMemcpyAsync(ho + total, ws.out_score.p, total * 4, hipMemcpyDeviceToHost, st));
            COBS_HIP(hipStreamSynchronize(st));
        }
        out.ids = ho;
        out.scores = ho + total;
        return COBS_OK;
    }
}

cobs_status reserve_workspace(cobs_index *ix, Workspace &ws, uint64_t W, uint32_t n,
                              hipStream_t st)
{
    // upper bounds of what run_batch asks for: query bytes <= W + n * q,
    // global dedup slots < 4 W + n (capacity < 4 windows, plus a flag word)
    const uint32_t h = ix->prm.num_hashes;
    const uint64_t nbytes = W + (uint64_t)n * ix->prm.q;
    const uint64_t n_slices = ix->slices.size();
    const size_t meta = batch_meta_bytes(n);
    COBS_HIP(ws.h_stage.ensure(meta + nbytes));
    COBS_HIP(ws.meta.ensure(meta));
    COBS_HIP(ws.bytes.ensure(nbytes + 64));
    COBS_HIP(ws.terms.ensure(std::max<uint64_t>(W, 1) * 8));
    COBS_HIP(ws.uterms.ensure(std::max<uint64_t>(W, 1) * 8));
    COBS_HIP(ws.hashes.ensure(std::max<uint64_t>(W, 1) * 8 * h));
    COBS_HIP(ws.head.ensure(sizeof(Scalars) + (size_t)n * 8 + (size_t)(n + 1) * 4));
    COBS_HIP(ws.table.ensure(std::max<uint64_t>(4 * W + n, 1) * 8));
    if (ws.tickets_slots < (uint64_t)n * n_slices || !ws.tickets.p) {
        COBS_HIP(ws.tickets.ensure(std::max<uint64_t>((uint64_t)n * n_slices, 1) * 4, true, st));
        ws.tickets_slots = ws.tickets.cap / 4;
    }
    COBS_HIP(ws.qinfo.ensure((size_t)n * sizeof(QInfo)));
    COBS_HIP(ws.chunk_prefix.ensure((size_t)(n + 1) * 4));
    COBS_HIP(ws.qorder.ensure((size_t)n * 4));
    COBS_HIP(ws.qcount.ensure((size_t)n * 4));
    ws.cand_cap = std::max<uint64_t>(ws.cand_cap, std::max<uint64_t>(1 << 20, (uint64_t)n * 64));
    COBS_HIP(ws.cand_key.ensure(ws.cand_cap * 8));
    COBS_HIP(ws.cand_q.ensure(ws.cand_cap * 4));
    COBS_HIP(ws.gstart.ensure((size_t)(n + 1) * 4));
    COBS_HIP(ws.gcursor.ensure((size_t)n * 4));
    COBS_HIP(ws.seg_a.ensure(ws.cand_cap * 8));
    COBS_HIP(ws.seg_b.ensure(ws.cand_cap * 8));
    COBS_HIP(ws.out_id.ensure(ws.cand_cap * 4));
    COBS_HIP(ws.out_score.ensure(ws.cand_cap * 4));
    COBS_HIP(ws.h_small.ensure(sizeof(Scalars) + (size_t)n * 8 + (size_t)(n + 1) * 4));
    COBS_HIP(ws.h_out.ensure(ws.cand_cap * 8));
    for (hipEvent_t &e : ws.ev)
        if (!e) COBS_HIP(hipEventCreate(&e));
    COBS_HIP(hipStreamSynchronize(st));
    return COBS_OK;
}

cobs_status make_hits(const BatchOut &o, uint32_t q0, uint32_t n, cobs_hits *dst)
{
    for (uint32_t i = 0; i < n; ++i) {
        cobs_hits &h = dst[i];
        const uint32_t k = o.n[q0 + i], s = o.start[q0 + i];
        h.n = k;
        h.num_terms = o.num_terms[q0 + i];
        h.doc_id = (uint32_t *)std::malloc(std::max<size_t>(k, 1) * 4);
        h.score = (uint32_t *)std::malloc(std::max<size_t>(k, 1) * 4);
        if (!h.doc_id || !h.score) return set_error(COBS_ENOMEM, "out of host memory");
        if (k) {
            std::memcpy(h.doc_id, o.ids + s, (size_t)k * 4);
            std::memcpy(h.score, o.scores + s, (size_t)k * 4);
        }
    }
    return COBS_OK;
}

}  // namespace cobs

extern "C" {

void cobs_hits_free(cobs_hits *hits, uint32_t n)
{
    if (!hits) return;
    for (uint32_t i = 0; i < n; ++i) {
        std::free(hits[i].doc_id);
        std::free(hits[i].score);
    }
    std::free(hits);
}

}  // extern "C"

struct cobs_results {
    std::vector<uint32_t> num_terms;
    std::vector<uint64_t> off;
    std::vector<uint32_t> ids, scores;
};

namespace {

// Batched: one pipeline run over all queries.  Plain: one run per query.
// sink(batch output, first query of the batch, queries in the batch).
template <typename Sink>
cobs_status query_driver(cobs_index *ix, const uint8_t *bytes, const uint64_t *q_off,
                         uint32_t n_queries, const cobs_query_opts *opts, void *stream, Sink sink)
{
    if (opts->mode != COBS_MODE_BATCHED && opts->mode != COBS_MODE_PLAIN)
        return set_error(COBS_EINVAL, "unknown mode");
    hipStream_t st = (hipStream_t)stream;
    Workspace *ws = acquire_workspace(ix);
    BatchSpec spec;
    spec.bytes = bytes;
    spec.mem = opts->mem;
    spec.k_num = opts->k_num;
    spec.k_den = opts->k_den;
    spec.topk = opts->topk;
    spec.score_bits = opts->score_bits;
    spec.chunk = opts->chunk;
    cobs_status s = COBS_OK;
    BatchOut bo;
    if (opts->mode == COBS_MODE_BATCHED) {
        spec.q_off = q_off;
        spec.n = n_queries;
        s = run_batch(ix, *ws, spec, st, bo);
        if (s == COBS_OK) s = sink(bo, 0u, n_queries);
    } else {
        for (uint32_t i = 0; i < n_queries && s == COBS_OK; ++i) {
            spec.q_off = q_off + i;
            spec.n = 1;
            s = run_batch(ix, *ws, spec, st, bo);
            if (s == COBS_OK) s = sink(bo, i, 1u);
        }
    }
    release_workspace(ix, ws);
    return s;
}

}  // namespace

extern "C" {

cobs_status cobs_query_batch(cobs_index *ix, const uint8_t *bytes, const uint64_t *q_off,
                             uint32_t n_queries, const cobs_query_opts *opts, void *stream,
                             cobs_hits **out)
{
    if (!ix || !opts || !out) return set_error(COBS_EINVAL, "NULL argument");
    *out = nullptr;
    cobs_hits *hits = (cobs_hits *)std::calloc(std::max<uint32_t>(n_queries, 1), sizeof(cobs_hits));
    if (!hits) return set_error(COBS_ENOMEM, "out of host memory");
    cobs_status s = query_driver(ix, bytes, q_off, n_queries, opts, stream,
                                 [&](const BatchOut &bo, uint32_t q0, uint32_t n) {
                                     return make_hits(bo, 0, n, hits + q0);
                                 });
    if (s != COBS_OK) {
        cobs_hits_free(hits, n_queries);
        return s;
    }
    *out = hits;
    return COBS_OK;
}

cobs_status cobs_query_results(cobs_index *ix, const uint8_t *bytes, const uint64_t *q_off,
                               uint32_t n_queries, const cobs_query_opts *opts, void *stream,
                               cobs_results **out)
{
    if (!ix || !opts || !out) return set_error(COBS_EINVAL, "NULL argument");
    *out = nullptr;
    auto *r = new cobs_results();
    r->num_terms.assign(n_queries, 0);
    r->off.assign((size_t)n_queries + 1, 0);
    cobs_status s = query_driver(ix, bytes, q_off, n_queries, opts, stream,
                                 [&](const BatchOut &bo, uint32_t q0, uint32_t n) {
                                     const uint64_t base = r->ids.size(), tot = bo.start[n];
                                     r->ids.insert(r->ids.end(), bo.ids, bo.ids + tot);
                                     r->scores.insert(r->scores.end(), bo.scores, bo.scores + tot);
                                     for (uint32_t i = 0; i < n; ++i) {
                                         r->num_terms[q0 + i] = bo.num_terms[i];
                                         r->off[q0 + i + 1] = base + bo.start[i + 1];
                                     }
                                     return COBS_OK;
                                 });
    if (s != COBS_OK) {
        delete r;
        return s;
    }
    *out = r;
    return COBS_OK;
}

cobs_status cobs_results_view(const cobs_results *r, uint32_t *n_queries,
                              const uint32_t **num_terms, const uint64_t **hit_off,
                              const uint32_t **doc_id, const uint32_t **score)
{
    if (!r) return set_error(COBS_EINVAL, "results is NULL");
    if (n_queries) *n_queries = (uint32_t)r->num_terms.size();
    if (num_terms) *num_terms = r->num_terms.data();
    if (hit_off) *hit_off = r->off.data();
    if (doc_id) *doc_id = r->ids.data();
    if (score) *score = r->scores.data();
    return COBS_OK;
}

void cobs_results_free(cobs_results *r) { delete r; }

cobs_status cobs_query_scores(cobs_index *ix, const uint8_t *bytes, const uint64_t *q_off,
                              uint32_t n_queries, uint32_t mem, void *stream, uint32_t *scores,
                              uint32_t *num_terms)
{
    if (!ix || (!scores && n_queries && ix->n_docs)) return set_error(COBS_EINVAL, "NULL argument");
    Workspace *ws = acquire_workspace(ix);
    BatchSpec spec;
    spec.bytes = bytes;
    spec.q_off = q_off;
    spec.n = n_queries;
    spec.mem = mem;
    spec.full_scores = scores ? scores : (uint32_t *)&spec;
    BatchOut bo;
    cobs_status s = run_batch(ix, *ws, spec, (hipStream_t)stream, bo);
    release_workspace(ix, ws);
    if (s == COBS_OK && num_terms) std::memcpy(num_terms, bo.num_terms.data(), (size_t)n_queries * 4);
    return s;
}

cobs_status cobs_query_terms(const cobs_index *cix, const uint8_t *bytes, const uint64_t *q_off,
                             uint32_t n_queries, uint32_t mem, void *stream, uint64_t *terms,
                             uint32_t *num_terms)
{
    cobs_index *ix = const_cast<cobs_index *>(cix);
    if (!ix || !terms) return set_error(COBS_EINVAL, "NULL argument");
    Workspace *ws = acquire_workspace(ix);
    BatchSpec spec;
    spec.bytes = bytes;
    spec.q_off = q_off;
    spec.n = n_queries;
    spec.mem = mem;
    spec.terms_out = terms;
    BatchOut bo;
    cobs_status s = run_batch(ix, *ws, spec, (hipStream_t)stream, bo);
    release_workspace(ix, ws);
    if (s == COBS_OK && num_terms) std::memcpy(num_terms, bo.num_terms.data(), (size_t)n_queries * 4);
    return s;
}

cobs_status cobs_set_tuning(cobs_index *ix, const cobs_tuning *t)
{
    if (!ix || !t) return set_error(COBS_EINVAL, "NULL argument");
    if (t->unroll && !gather_unroll_valid((int)t->unroll, (int)ix->prm.num_hashes))
        return set_error(COBS_EINVAL, "unsupported unroll for this index");
    ix->tuned_unroll = (int)t->unroll;
    ix->tuned_chunk = t->chunk;
    return COBS_OK;
}

cobs_status cobs_tune(cobs_index *ix, const uint8_t *bytes, const uint64_t *q_off,
                      uint32_t n_queries, uint32_t mem, void *stream, cobs_tuning *best)
{
    if (!ix || !best) return set_error(COBS_EINVAL, "NULL argument");
    const int h = (int)ix->prm.num_hashes;
    const int unrolls[2] = {h == 1 ? 4 : 2, h == 1 ? 8 : 4};
    const uint32_t chunks[] = {0, 512, 1024, 2048, 4096, 8192, 16384, 1u << 20};
    Workspace *ws = acquire_workspace(ix);
    cobs_tuning win{0, 0, 1e300};
    cobs_status s = COBS_OK;
    for (int u : unrolls) {
        for (uint32_t c : chunks) {
            BatchSpec spec;
            spec.bytes = bytes;
            spec.q_off = q_off;
            spec.n = n_queries;
            spec.mem = mem;
            spec.k_num = 1;
            spec.k_den = 1;
            spec.unroll = (uint32_t)u;
            spec.chunk_cap = c;
            spec.time_gather = true;
            double t = 1e300;
            for (int rep = 0; rep < 2 && s == COBS_OK; ++rep) {   // first run warms up
                BatchOut bo;
                s = run_batch(ix, *ws, spec, (hipStream_t)stream, bo);
                if (rep) t = bo.gather_ms;
            }
            if (s != COBS_OK) break;
            if (t < win.gather_ms) win = cobs_tuning{(uint32_t)u, c, t};
        }
    }
    release_workspace(ix, ws);
    if (s != COBS_OK) return s;
    ix->tuned_unroll = (int)win.unroll;
    ix->tuned_chunk = win.chunk;
    *best = win;
    return COBS_OK;
}

cobs_status cobs_profile(int enable)
{
    g_prof.store(enable ? 1 : 0);
    return COBS_OK;
}

cobs_status cobs_profile_read(cobs_kernel_timing *gather, int reset)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (gather) *gather = g_prof_acc;
    if (reset) g_prof_acc = cobs_kernel_timing{};
    return COBS_OK;
}

}  // extern "C"
