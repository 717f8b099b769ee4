// Index operations beyond building and querying: out-of-core residency
// (cobs_index_offload / onload), index files (cobs_index_save / load) and
// merging (cobs_index_merge), following section 2.3 of the COBS paper.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "runtime.h"

using namespace cobs;

extern "C" {

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
        if (stage) COBS_HIP(dev_alloc(&ix->d_stage[i], stage));
        COBS_HIP(hipEventCreateWithFlags(&ix->ev_copy[i], hipEventDisableTiming));
        COBS_HIP(hipEventCreateWithFlags(&ix->ev_done[i], hipEventDisableTiming));
    }
    COBS_HIP(hipStreamCreateWithFlags(&ix->copy_stream, hipStreamNonBlocking));
    COBS_HIP(dev_alloc(&ix->d_group_slices, std::max<size_t>(rebased.size(), 1) * sizeof(SliceDesc)));
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
    hipError_t e = hipHostMalloc((void **)&ix->h_matrix, std::max<uint64_t>(ix->total_bytes, 1),
                                 hipHostMallocMapped);
    if (e != hipSuccess) {
        ix->h_matrix = nullptr;
        return set_error(COBS_ENOMEM, "pinned host memory for the matrix");
    }
    if ((e = hipHostGetDevicePointer((void **)&ix->h_dev_matrix, ix->h_matrix, 0)) != hipSuccess) {
        ix->release_offload();
        return hip_error(e, "hipHostGetDevicePointer(matrix)");
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
    dev_free(ix->d_matrix);
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
        if (hipHostMalloc((void **)&ix->h_matrix, std::max<uint64_t>(T, 1), hipHostMallocMapped) != hipSuccess) {
            ix->h_matrix = nullptr;
            return set_error(COBS_ENOMEM, "pinned host memory for the matrix");
        }
        if (hipHostGetDevicePointer((void **)&ix->h_dev_matrix, ix->h_matrix, 0) != hipSuccess)
            return set_error(COBS_EDEVICE, "hipHostGetDevicePointer(matrix)");
        if (T && std::fread(ix->h_matrix, 1, T, in.f) != T) return bad("truncated matrix");
        if ((s = setup_staging(ix.get(), groups, stage)) != COBS_OK) return s;
    } else {
        if (T) {
            if (dev_alloc(&ix->d_matrix, T) != hipSuccess)
                return set_error(COBS_ENOMEM, "device memory for the matrix");
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
        if (dev_alloc(&ix->d_matrix, ix->total_bytes) != hipSuccess)
            return set_error(COBS_ENOMEM, "device memory for the matrix");
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
    hipError_t e = dev_alloc(&d, std::max<uint64_t>(ix->total_bytes, 1));
    if (e != hipSuccess) return set_error(COBS_ENOMEM, "device memory for the matrix");
    if (ix->total_bytes && (e = hipMemcpy(d, ix->h_matrix, ix->total_bytes, hipMemcpyHostToDevice)) != hipSuccess) {
        dev_free(d);
        return hip_error(e, "hipMemcpy(matrix to device)");
    }
    ix->d_matrix = d;
    ix->release_offload();
    return COBS_OK;
}

}  // extern "C"
