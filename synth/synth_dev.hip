// Device twin of synth.c's document-bases generator: Philox4x32-10 (Salmon et
// al., SC 2011) addressed by (64-base word, document, stream 2) under the
// workload seed, so documents of the large workloads can be written straight
// into HBM.  Must stay bit-identical to synth_doc_bases() in synth.c.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint32_t kStreamDocBases = 2;

__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// one workgroup per document; each thread writes 64 bases per Philox call
__global__ void doc_bases_kernel(uint64_t seed, const uint64_t *off, uint32_t first,
                                 uint8_t *out)
{
    const uint32_t d = blockIdx.x;
    const uint64_t begin = off[d], len = off[d + 1] - begin;
    const uint64_t words = (len + 63) / 64;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const char acgt[4] = {'A', 'C', 'G', 'T'};
    for (uint64_t w = threadIdx.x; w < words; w += blockDim.x) {
        uint32_t c[4] = {(uint32_t)w, (uint32_t)(w >> 32), first + d, kStreamDocBases};
        philox10(c, k0, k1);
        uint8_t *dst = out + begin + w * 64;
        const uint64_t n = (len - w * 64) < 64 ? (len - w * 64) : 64;
        if (n == 64 && ((uintptr_t)dst & 15) == 0) {
            uint32_t packed[16];
            for (int j = 0; j < 16; ++j) {
                uint32_t v = 0;
                for (int b = 0; b < 4; ++b) {
                    int i = j * 4 + b;
                    v |= (uint32_t)(uint8_t)acgt[(c[i >> 4] >> (2 * (i & 15))) & 3] << (8 * b);
                }
                packed[j] = v;
            }
            uint4 *d4 = reinterpret_cast<uint4 *>(dst);
            for (int j = 0; j < 4; ++j)
                d4[j] = make_uint4(packed[4 * j], packed[4 * j + 1], packed[4 * j + 2],
                                   packed[4 * j + 3]);
        } else {
            for (uint64_t i = 0; i < n; ++i)
                dst[i] = (uint8_t)acgt[(c[i >> 4] >> (2 * (i & 15))) & 3];
        }
    }
}

}  // namespace

// Documents [first, first+count): bases written at out + off[d] (device
// pointers; off holds count+1 offsets).  Returns 0 or a hipError_t.
extern "C" int synth_dev_doc_bases(uint64_t seed, const uint64_t *off, uint32_t first,
                                   uint32_t count, uint8_t *out, void *stream)
{
    if (count == 0) return 0;
    hipLaunchKernelGGL(doc_bases_kernel, dim3(count), dim3(256), 0, (hipStream_t)stream,
                       seed, off, first, out);
    return (int)hipGetLastError();
}
