// The gather kernel of the COBS query path (section 2.2 of the COBS paper):
// row gather, AND, ADD and report.  Persistent wavefronts take work items
// (query chunk, column slice), fetch the h rows of every term of the chunk
// (one coalesced 1 KiB line per row slice, or several terms per load for
// narrow slices), AND them, add the surviving bits into bit-plane counters
// held in VGPRs, merge the counts of split queries in a score buffer, and
// report each slice of a query: full scores, or the documents reaching the
// threshold (top-k by a bit-plane radix select).
#include "kernels.h"

#include <hip/hip_runtime.h>

#include "device_util.h"

namespace cobs {
namespace {

// ---- gather / AND / ADD / threshold-or-top-k ---------------------------------------------

// Chunks of a query in the first of two pruning launches: the fraction
// f = f0 + fz / sqrt(l) of its nch chunks, rounded up, at least 1; all of
// them (nothing left to prune) when f >= 0.9.
__device__ __forceinline__ uint32_t phase1_chunks(uint32_t nch, uint32_t ell, float f0, float fz)
{
    const float f = f0 + fz * rsqrtf((float)(ell > 1u ? ell : 1u));
    if (!(f < 0.9f)) return nch;
    const uint32_t n1 = (uint32_t)ceilf(f * (float)nch);
    return n1 < 1u ? 1u : (n1 > nch ? nch : n1);
}

// full adder on 32 independent bit positions: a + b + c = s + 2 carry
__device__ __forceinline__ void csa(uint32_t &s, uint32_t &carry, uint32_t a, uint32_t b, uint32_t c)
{
    const uint32_t u = a ^ b;
    s = u ^ c;
    carry = (a & b) | (u & c);
}

// Bit-sliced per-document counters of one wavefront slice: plane p holds bit
// p of the score of every document; each lane owns 4 dwords = 128 documents.
// A group of U indicator vectors is added through a carry-save adder tree
// (ones, twos, fours planes absorb the inputs), and only the tree's single
// carry vector ripples into the higher planes.
template <int P>
struct Counter {
    uint32_t H[P][4];

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int d = 0; d < 4; ++d) H[p][d] = 0;
    }

    __device__ __forceinline__ void ripple(int d, int from, uint32_t c)
    {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (p < from) continue;
            const uint32_t h = H[p][d];
            H[p][d] = h ^ c;
            c = h & c;
        }
    }

    // add U (1, 2, 4, 8 or 16) indicator vectors
    template <int U>
    __device__ __forceinline__ void add(const u32x4 *x)
    {
        if constexpr (U == 16) {
            add<8>(x);
            add<8>(x + 8);
            return;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t xs[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xs[u] = x[u][d];
            if constexpr (U == 1) {
                ripple(d, 0, xs[0]);
            } else if constexpr (U == 2) {
                uint32_t t0;
                csa(H[0][d], t0, H[0][d], xs[0], xs[1]);
                ripple(d, 1, t0);
            } else if constexpr (U == 4) {
                uint32_t t0, t1, e;
                csa(H[0][d], t0, H[0][d], xs[0], xs[1]);
                csa(H[0][d], t1, H[0][d], xs[2], xs[3]);
                csa(H[1][d], e, H[1][d], t0, t1);
                ripple(d, 2, e);
            } else {
                static_assert(U == 8 || U == 16, "U must be 1, 2, 4, 8 or 16");
                uint32_t t0, t1, t2, t3, u0, u1, e;
                csa(H[0][d], t0, H[0][d], xs[0], xs[1]);
                csa(H[0][d], t1, H[0][d], xs[2], xs[3]);
                csa(H[1][d], u0, H[1][d], t0, t1);
                csa(H[0][d], t2, H[0][d], xs[4], xs[5]);
                csa(H[0][d], t3, H[0][d], xs[6], xs[7]);
                csa(H[1][d], u1, H[1][d], t2, t3);
                csa(H[2][d], e, H[2][d], u0, u1);
                ripple(d, 3, e);
            }
        }
    }

    // documents with score >= T (T < 2^P)
    __device__ __forceinline__ void ge(uint32_t T, uint32_t out[4]) const
    {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t gt = 0, eq = ~0u;
#pragma unroll
            for (int p = P - 1; p >= 0; --p) {
                if ((T >> p) & 1u) {
                    eq &= H[p][d];
                } else {
                    gt |= eq & H[p][d];
                    eq &= ~H[p][d];
                }
            }
            out[d] = gt | eq;
        }
    }

    __device__ __forceinline__ uint32_t score(int d, int bit) const
    {
        uint32_t s = 0;
#pragma unroll
        for (int p = 0; p < P; ++p) s |= ((H[p][d] >> bit) & 1u) << p;
        return s;
    }
};

// Whether any document of a split (query, slice) has a count of at least
// need in its score buffer (lanes below L).  Layout: while l < 2^16, four
// 16-bit counts per 64-bit word, 32 words per lane at i*L + lane; else one
// 32-bit count per document, 128 per lane at i*L + lane.
__device__ __forceinline__ bool any_count_reaches(const uint32_t *acc, uint32_t L, uint32_t lane,
                                                  bool packed, uint32_t need)
{
    bool any = false;
    if (lane >= L) return false;
    if (packed) {
        const unsigned long long *acc4 = (const unsigned long long *)acc;
#pragma unroll 4
        for (uint32_t i = 0; i < 32; ++i) {
            const unsigned long long v = __hip_atomic_load(acc4 + i * L + lane, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int j = 0; j < 4; ++j) any |= ((uint32_t)(v >> (16 * j)) & 0xFFFFu) >= need;
        }
    } else {
#pragma unroll 4
        for (uint32_t i = 0; i < 128; ++i)
            any |= __hip_atomic_load(acc + i * L + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
    }
    return any;
}

// U: terms whose rows are in flight per wavefront (h rows each).  Kernels
// with several hashes and at most 12 counter planes are held to 128 VGPRs
// (4 wavefronts per SIMD instead of 3; no spills): the text index's gather,
// bound by L2-miss reads, ran 3% faster with the extra wavefront.
// kPacked: every slice of the launch is narrow (at most 512 bytes wide); G =
// 2, 4 or 8 terms share one load, 64 / G lanes each, and the G partial
// counts of every document are summed at the end of the item.
template <int P, int U, bool kH1, bool kPacked>
__global__ __launch_bounds__(256, (kH1 || P > 12) ? 1 : 4) void gather_kernel(GatherArgs a)
{
    const uint32_t lane = lane_id();
    const uint32_t n_chunks = a.chunk_prefix[a.n_queries];
    const uint64_t total = (uint64_t)n_chunks * a.n_slices;
    // item = major * minor_count + minor
    const uint32_t minor_count = a.slice_major ? n_chunks : a.n_slices;
    Counter<P> cnt;

    for (;;) {
        uint64_t item = 0;
        if (lane == 0) item = atomicAdd(a.work_counter, 1ull);
        item = bcast64(item);
        if (item >= total) break;
        // chunks in query-size order; the slices of one chunk side by side,
        // or one slice at a time (its rows then stay in the last-level cache)
        const uint32_t major = (uint32_t)(item / minor_count);
        const uint32_t minor = (uint32_t)(item - (uint64_t)major * minor_count);
        const uint32_t c = a.slice_major ? minor : major;
        const uint32_t sl = a.slice_major ? major : minor;
        const uint32_t rank = bsearch_le(a.chunk_prefix, a.n_queries, c);
        const uint32_t qi = a.qorder[rank];
        const uint32_t chunk = c - a.chunk_prefix[rank];
        const QInfo qn = a.qinfo[qi];
        const SliceDesc sd = a.slices[sl];
        // two launches for split queries under pruning: phase 1 takes the
        // first n1 chunks of every query, phase 2 the others, which skip
        // their terms where phase 1 found that no document of the slice can
        // reach T any more
        const uint32_t n1 = a.phase ? phase1_chunks(qn.nch, qn.ell, a.phase1_f0, a.phase1_fz) : qn.nch;
        if (a.phase && (a.phase == 1) != (chunk < n1)) continue;
        const bool dead = a.phase == 2 && __hip_atomic_load(&a.dead[(uint64_t)qi * a.n_slices + sl],
                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        const uint32_t kbeg = chunk * a.chunk;
        const uint32_t kend = dead ? kbeg : min(qn.ell, kbeg + a.chunk);
        // uniform slice geometry in SGPRs
        const uint64_t sbase = bcast64(sd.base);
        const uint32_t sstride = uniform_u32(sd.stride);
        const uint32_t srows = uniform_u32(sd.rows);
        const uint32_t swidth = uniform_u32(sd.width);
        // lanes per term (lpt) and this lane's term group and column; every
        // lane loads (no divergent loads: they serialise the memory pipeline);
        // lanes past the slice width read an in-row address and mask the
        // bits off
        uint32_t lpt = 64u, grp = 0u, col = lane;
        if constexpr (kPacked) {
            lpt = swidth <= 128u ? 8u : (swidth <= 256u ? 16u : 32u);
            grp = lane / lpt;
            col = lane & (lpt - 1u);
        }
        const uint32_t loff = min(col * 16u, swidth - 16u);
        const uint32_t lmask = col * 16u < swidth ? ~0u : 0u;
        const uint8_t *mrow0 = a.matrix + sbase + loff;
        const uint64_t *hp = a.hashes + qn.hbase * a.h;

        cnt.clear();
        // pruning (unpacked launches): after every 64 terms the item ends if
        // every document of the slice scores below T minus the terms not yet
        // counted (in this chunk or any other): none of them can reach T any
        // more, and their partial counts stay below T, so the reported hits
        // and scores do not change.  (A per-lane stop would also spare the
        // lines of dead lanes in a live slice, but its predicated loads cost
        // this kernel its fourth wavefront per SIMD.)
        const bool prune = !kPacked && a.prune != 0;
        for (uint32_t k0 = kbeg; k0 < kend; k0 += 64) {
            if (prune && k0 > kbeg) {
                const uint32_t left = qn.ell - (k0 - kbeg);
                if (qn.thr > left) {
                    uint32_t g[4];
                    cnt.ge(qn.thr - left, g);
                    if (__ballot((g[0] | g[1] | g[2] | g[3]) != 0u) == 0) break;
                }
            }
            const uint32_t n = min(64u, kend - k0);
            uint32_t r[kH1 ? 1 : kMaxHashes];
            if (lane < n) {
                if (kH1) {
                    r[0] = (uint32_t)(hp[k0 + lane] % srows);
                } else {
#pragma unroll
                    for (int i = 0; i < kMaxHashes; ++i)
                        if (i < (int)a.h) r[i] = (uint32_t)(hp[(uint64_t)(k0 + lane) * a.h + i] % srows);
                }
            }
            if constexpr (kPacked) {
                // group g takes terms j + g, j + G + g, ...; terms past n
                // repeat the last row and are masked off
                const uint32_t G = 64u / lpt;
                for (uint32_t j = 0; j < n; j += G * U) {
                    u32x4 v[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const uint32_t t = min(j + G * (uint32_t)u + grp, n - 1);
                        v[u] = load_row<kH1>(mrow0 + (uint64_t)(uint32_t)__shfl((int)r[0], (int)t, 64) * sstride);
                        if (!kH1) {
#pragma unroll
                            for (int i = 1; i < kMaxHashes; ++i)
                                if (i < (int)a.h)
                                    v[u] &= load_row<kH1>(
                                        mrow0 + (uint64_t)(uint32_t)__shfl((int)r[i], (int)t, 64) * sstride);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int u = 0; u < U; ++u) v[u] &= (j + G * (uint32_t)u + grp < n) ? lmask : 0u;
                    cnt.template add<U>(v);
                }
                continue;
            }
            for (uint32_t j = 0; j < n; j += U) {
                // a short last group repeats its last row (already in flight,
                // served by the cache) and masks the repeats off
                const uint32_t rem = n - j;
                u32x4 v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t t = j + min((uint32_t)u, rem - 1);
                    v[u] = load_row<kH1>(mrow0 + (uint64_t)lane_u32(r[0], t) * sstride);
                    if (!kH1) {
#pragma unroll
                        for (int i = 1; i < kMaxHashes; ++i)
                            if (i < (int)a.h)
                                v[u] &= load_row<kH1>(mrow0 + (uint64_t)lane_u32(r[i], t) * sstride);
                    }
                }
                // all U row loads in flight before the first is consumed
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] &= ((uint32_t)u < rem) ? lmask : 0u;
                cnt.template add<U>(v);
            }
        }

        // packed: lanes c, c + lpt, c + 2 lpt, ... hold partial counts of the
        // same 128 documents; butterfly rounds of bit-plane additions leave
        // the sums in every lane, then lanes from lpt on drop theirs (each
        // partial count is at most l < 2^P, so no carry leaves plane P - 1)
        if constexpr (kPacked) {
            for (uint32_t m = 32u; m >= lpt; m >>= 1) {
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    uint32_t carry = 0;
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const uint32_t x = cnt.H[p][d];
                        const uint32_t y = (uint32_t)__shfl_xor((int)x, (int)m, 64);
                        cnt.H[p][d] = x ^ y ^ carry;
                        carry = (x & y) | (carry & (x ^ y));
                    }
                }
            }
            if (lane >= lpt) cnt.clear();
        }

        // Several chunks of one (query, slice): each adds its counts into the
        // query's score buffer with device-scope atomic adds, then takes a
        // ticket; the last chunk to finish reads the totals back into bit
        // planes, clears the buffer for the next batch and reports.  The merge
        // costs the same for 2 chunks or 2,000.  Layout per slice: document
        // (lane, d, bit) at (d*32 + bit)*lanes + lane, or, while l < 2^16 (no
        // count can pass 16 bits), four documents (bit, bit+8, bit+16, bit+24)
        // in one 64-bit word at (d*8 + bit)*lanes + lane; either way one
        // instruction's lanes touch consecutive words.  Lanes past the slice's
        // documents hold zero counts and touch nothing.  Every access to the
        // buffer and the tickets is a device-scope atomic, so ordering needs
        // only the wait for this wavefront's adds before its ticket (no cache
        // write-back or invalidation).
        if (qn.nch > 1) {
            const uint32_t L = uniform_u32(sd.lanes);
            uint32_t *acc = a.accum + (uint64_t)qn.pbase * a.acc_words + uniform_u32(sd.acc_off);
            unsigned long long *acc4 = (unsigned long long *)acc;
            const bool packed = qn.ell < 65536u;
            if (packed) {
#pragma unroll
                for (int d = 0; d < 4; ++d) {
#pragma unroll 2
                    for (int b = 0; b < 8; ++b) {
                        const unsigned long long v =
                            (unsigned long long)cnt.score(d, b) |
                            ((unsigned long long)cnt.score(d, b + 8) << 16) |
                            ((unsigned long long)cnt.score(d, b + 16) << 32) |
                            ((unsigned long long)cnt.score(d, b + 24) << 48);
                        if (v)
                            __hip_atomic_fetch_add(acc4 + (d * 8 + b) * L + lane, v, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            } else {
#pragma unroll
                for (int d = 0; d < 4; ++d) {
#pragma unroll 4
                    for (int bit = 0; bit < 32; ++bit) {
                        const uint32_t c = cnt.score(d, bit);
                        if (c)
                            __hip_atomic_fetch_add(acc + (d * 32 + bit) * L + lane, c, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            }
            __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");   // adds done before the ticket
            const uint64_t slot = (uint64_t)qi * a.n_slices + sl;
            uint32_t *ticket = &a.tickets[slot];
            uint32_t tk = 0;
            if (lane == 0) tk = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tk = uniform_u32(tk);
            if (tk != qn.nch - 1) {
                // the last chunk of phase 1 (when phase 2 has chunks left):
                // after the first n1 chunks' c1 terms a document can still
                // gain l - c1; it marks the (query, slice) dead if no
                // document can reach T
                if (a.phase == 1 && tk == n1 - 1) {
                    const uint64_t c1 = min((uint64_t)qn.ell, (uint64_t)n1 * a.chunk);
                    const uint32_t left = qn.ell - (uint32_t)c1;
                    if (qn.thr > left && __ballot(any_count_reaches(acc, L, lane, packed, qn.thr - left)) == 0 &&
                        lane == 0)
                        __hip_atomic_store(&a.dead[slot], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                continue;
            }
            if (lane == 0) {
                __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (a.phase == 2) __hip_atomic_store(&a.dead[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            cnt.clear();
            if (lane < L) {
                if (packed) {
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
#pragma unroll 2
                        for (int b = 0; b < 8; ++b) {
                            unsigned long long *cell = acc4 + (d * 8 + b) * L + lane;
                            const unsigned long long v =
                                __hip_atomic_exchange(cell, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const uint32_t c = (uint32_t)(v >> (16 * j)) & 0xFFFFu;
#pragma unroll
                                for (int p = 0; p < P; ++p) cnt.H[p][d] |= ((c >> p) & 1u) << (b + 8 * j);
                            }
                        }
                    }
                } else {
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
#pragma unroll 4
                        for (int bit = 0; bit < 32; ++bit) {
                            const uint32_t c = __hip_atomic_exchange(acc + (d * 32 + bit) * L + lane, 0u,
                                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                            for (int p = 0; p < P; ++p) cnt.H[p][d] |= ((c >> p) & 1u) << bit;
                        }
                    }
                }
            }
        }

        // report this slice of the query
        uint32_t valid[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t b0 = lane * 128u + d * 32u;
            valid[d] = b0 >= sd.ndocs ? 0u : (sd.ndocs - b0 >= 32 ? ~0u : ((1u << (sd.ndocs - b0)) - 1u));
        }
        if (a.full_scores) {
            uint32_t *fs = a.full_scores + (uint64_t)qi * a.n_docs;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                uint32_t m = valid[d];
                while (m) {
                    const int bit = __builtin_ctz(m);
                    m &= m - 1;
                    fs[a.order[sd.doc0 + lane * 128u + d * 32u + bit]] = cnt.score(d, bit);
                }
            }
            continue;
        }
        if (qn.thr > qn.ell) continue;
        uint32_t M[4];
        cnt.ge(qn.thr, M);
#pragma unroll
        for (int d = 0; d < 4; ++d) M[d] &= valid[d];
        if (a.topk) {
            const uint32_t have = wave_sum(__popc(M[0]) + __popc(M[1]) + __popc(M[2]) + __popc(M[3]));
            if (have > a.topk) {
                // MSB-first radix select of the topk-th largest score among M
                uint32_t pre[4] = {M[0], M[1], M[2], M[3]};
                uint32_t need = a.topk, s = 0;
#pragma unroll
                for (int p = P - 1; p >= 0; --p) {
                    const uint32_t c1 = wave_sum(__popc(pre[0] & cnt.H[p][0]) + __popc(pre[1] & cnt.H[p][1]) +
                                                 __popc(pre[2] & cnt.H[p][2]) + __popc(pre[3] & cnt.H[p][3]));
                    if (c1 >= need) {
#pragma unroll
                        for (int d = 0; d < 4; ++d) pre[d] &= cnt.H[p][d];
                        s |= 1u << p;
                    } else {
                        need -= c1;
#pragma unroll
                        for (int d = 0; d < 4; ++d) pre[d] &= ~cnt.H[p][d];
                    }
                }
                uint32_t G[4];
                cnt.ge(s, G);
#pragma unroll
                for (int d = 0; d < 4; ++d) M[d] &= G[d];
            }
        }
        const uint32_t mine_n = __popc(M[0]) + __popc(M[1]) + __popc(M[2]) + __popc(M[3]);
        const uint32_t tot = wave_sum(mine_n);
        if (tot == 0) continue;
        uint64_t base = 0;
        if (lane == 0) {
            base = atomicAdd(a.cand_counter, (unsigned long long)tot);
            atomicAdd(&a.qcount[qi], tot);
        }
        base = bcast64(base);
        uint64_t pos = base + wave_excl_scan(mine_n);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t m = M[d];
            while (m) {
                const int bit = __builtin_ctz(m);
                m &= m - 1;
                if (pos < a.cand_cap) {
                    const uint32_t id = a.order[sd.doc0 + lane * 128u + d * 32u + bit];
                    a.cand_key[pos] = ((uint64_t)cnt.score(d, bit) << 32) | (uint32_t)~id;
                    a.cand_q[pos] = qi;
                }
                ++pos;
            }
        }
    }
}

// Instantiated variants: h = 1 with 4 or 8 terms in flight (and 16 for the
// unpacked kernel, which single short queries use), h > 1 with 2 or 4 (each
// term then has h rows in flight).
template <int P, bool kPacked>
hipError_t launch_gather_pk(const GatherArgs &a, int unroll, int grid, hipStream_t st)
{
    if (a.h == 1) {
        if constexpr (!kPacked) {
            if (unroll == 16) {
                hipLaunchKernelGGL((gather_kernel<P, 16, true, false>), dim3(grid), dim3(256), 0, st, a);
                return hipGetLastError();
            }
        }
        if (unroll == 8)
            hipLaunchKernelGGL((gather_kernel<P, 8, true, kPacked>), dim3(grid), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((gather_kernel<P, 4, true, kPacked>), dim3(grid), dim3(256), 0, st, a);
    } else {
        if (unroll == 4)
            hipLaunchKernelGGL((gather_kernel<P, 4, false, kPacked>), dim3(grid), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((gather_kernel<P, 2, false, kPacked>), dim3(grid), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

template <int P>
hipError_t launch_gather_p(const GatherArgs &a, int unroll, int grid, bool packed, hipStream_t st)
{
    return packed ? launch_gather_pk<P, true>(a, unroll, grid, st)
                  : launch_gather_pk<P, false>(a, unroll, grid, st);
}

template <int P, bool kPacked>
int occ_of_pk(int unroll, int h)
{
    int blocks = 0;
    hipError_t e;
    if (h == 1 && unroll == 16 && !kPacked)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gather_kernel<P, 16, true, false>, 256, 0);
    else if (h == 1)
        e = unroll == 8
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gather_kernel<P, 8, true, kPacked>, 256, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gather_kernel<P, 4, true, kPacked>, 256, 0);
    else
        e = unroll == 4
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gather_kernel<P, 4, false, kPacked>, 256, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, gather_kernel<P, 2, false, kPacked>, 256, 0);
    if (e != hipSuccess || blocks < 1) blocks = 1;
    return blocks;
}

template <int P>
int occ_of_p(int unroll, int h, bool packed)
{
    return packed ? occ_of_pk<P, true>(unroll, h) : occ_of_pk<P, false>(unroll, h);
}

}  // namespace

int gather_planes_for(uint64_t max_terms)
{
    int bits = 0;
    while (bits < 64 && (max_terms >> bits) != 0) ++bits;
    for (int p : {8, 10, 12, 14, 16, 20, 24})
        if (bits <= p) return p;
    return 32;
}

int gather_default_unroll(int h) { return h == 1 ? 8 : 2; }

bool gather_unroll_valid(int unroll, int h)
{
    return h == 1 ? (unroll == 4 || unroll == 8) : (unroll == 2 || unroll == 4);
}

hipError_t launch_gather(const GatherArgs &a, int planes, int unroll, int grid, bool packed,
                         hipStream_t st)
{
    switch (planes) {
    case 8: return launch_gather_p<8>(a, unroll, grid, packed, st);
    case 10: return launch_gather_p<10>(a, unroll, grid, packed, st);
    case 12: return launch_gather_p<12>(a, unroll, grid, packed, st);
    case 14: return launch_gather_p<14>(a, unroll, grid, packed, st);
    case 16: return launch_gather_p<16>(a, unroll, grid, packed, st);
    case 20: return launch_gather_p<20>(a, unroll, grid, packed, st);
    case 24: return launch_gather_p<24>(a, unroll, grid, packed, st);
    case 32: return launch_gather_p<32>(a, unroll, grid, packed, st);
    default: return hipErrorInvalidValue;
    }
}

int gather_grid(int planes, int unroll, int h, bool packed)
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
    }
    int occ = 1;
    switch (planes) {
    case 8: occ = occ_of_p<8>(unroll, h, packed); break;
    case 10: occ = occ_of_p<10>(unroll, h, packed); break;
    case 12: occ = occ_of_p<12>(unroll, h, packed); break;
    case 14: occ = occ_of_p<14>(unroll, h, packed); break;
    case 16: occ = occ_of_p<16>(unroll, h, packed); break;
    case 20: occ = occ_of_p<20>(unroll, h, packed); break;
    case 24: occ = occ_of_p<24>(unroll, h, packed); break;
    default: occ = occ_of_p<32>(unroll, h, packed); break;
    }
    return cus * occ;
}

}  // namespace cobs
