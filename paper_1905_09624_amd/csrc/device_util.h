// Wavefront helpers shared by the HIP kernels of the library (gfx950:
// 64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cobs {
namespace {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One lane's 16 bytes of a row slice.  With one hash per term a row is read
// once per (term, query) from an index far larger than the caches, so the
// read does not displace cached data (non-temporal); with several hashes per
// term (the small text index) ordinary loads let the caches serve repeats,
// which measured 13% faster there and 10% slower on the 54 GB DNA index.
template <bool kNonTemporal>
__device__ __forceinline__ u32x4 load_row(const uint8_t *p)
{
    if constexpr (kNonTemporal) return __builtin_nontemporal_load((const u32x4 *)p);
    else return *(const u32x4 *)p;
}

// The lane builtins return int: convert to uint32_t before any widening, or
// a value with bit 31 set is sign-extended into the upper word.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

__device__ __forceinline__ uint32_t lane_u32(uint32_t v, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}

__device__ __forceinline__ uint64_t bcast64(uint64_t v)
{
    const uint32_t lo = uniform_u32((uint32_t)v);
    const uint32_t hi = uniform_u32((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// sum over the 64 lanes (every lane must be active); result is uniform
__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return uniform_u32(v);
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v)
{
    const uint32_t lane = lane_id();
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    return x - v;
}

// largest i in [0, n) with a[i] <= v, given a[0] <= v < a[n]
template <typename T>
__device__ __forceinline__ uint32_t bsearch_le(const T *a, uint32_t n, uint64_t v)
{
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)a[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// bsearch_le for a value v uniform over the wavefront (every lane active): 64
// probes per step, so three steps cover 10^5 entries.
template <typename T>
__device__ __forceinline__ uint32_t wave_search_le(const T *a, uint32_t n, uint64_t v)
{
    const uint32_t lane = lane_id();
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t i = lo + lane * step;
        const uint64_t m = __ballot(i < hi && (uint64_t)a[i] <= v);   // lanes 0 .. k-1
        const uint32_t k = 64u - (uint32_t)__builtin_clzll(m);
        const uint32_t nhi = lo + k * step;
        lo += (k - 1) * step;
        if (nhi < hi) hi = nhi;
    }
    return lo;
}

}  // namespace
}  // namespace cobs
