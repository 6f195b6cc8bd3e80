// Deferred binning of samples (Fig. 2 step 3): the sweep kernel stores each
// sample's bin index alpha * 2^K + phi as a 32-bit key, and these kernels count
// the keys into the circuit's histogram through LDS.  Histograms of more
// than 2^15 bins are cut into 2^15-bin buckets: workgroup (slab, bucket)
// reads its slab of keys, counts the keys of its bucket in LDS and writes
// the bucket's counts to its own partial row (no atomics in HBM); a second
// kernel adds the partial rows into the histogram with coalesced accesses.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "keyhist.h"

namespace pbit {

namespace {

constexpr uint32_t LDS_BITS = 15;
constexpr uint32_t BLOCK = 1024;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void count_key(uint32_t *h, uint32_t key, uint32_t lb, uint32_t b) {
    if ((key >> lb) == b) atomicAdd(&h[key & ((1u << lb) - 1u)], 1u);
}

// grid: S * NB workgroups, S a multiple of 8.  Workgroup w runs on XCD w % 8;
// the NB bucket workgroups of one slab go to the same XCD, one after the
// other, so they read the slab at about the same time through that XCD's L2.
__global__ void __launch_bounds__(BLOCK) keyhist_kernel(const uint32_t *__restrict__ keys, uint64_t M,
                                                       uint32_t bits, uint64_t slab, uint32_t *__restrict__ part) {
    __shared__ uint32_t h[1u << LDS_BITS];
    const uint32_t lb = bits < LDS_BITS ? bits : LDS_BITS;
    const uint32_t NB = 1u << (bits - lb);
    const uint32_t w = blockIdx.x, xcd = w & 7u, j = w >> 3;
    const uint32_t s = (j / NB) * 8u + xcd, b = j % NB;
    for (uint32_t i = threadIdx.x; i < (1u << lb); i += BLOCK) h[i] = 0u;
    __syncthreads();
    const uint64_t k0 = (uint64_t)s * slab;
    const uint64_t k1 = k0 + slab < M ? k0 + slab : M;
    if (k0 < k1) {
        // slab is a multiple of 4 and keys 16-byte aligned: whole vectors,
        // then the tail of the last slab
        const uint64_t v0 = k0 >> 2, v1 = k1 >> 2;
        const u32x4 *kv = (const u32x4 *)keys;
        for (uint64_t v = v0 + threadIdx.x; v < v1; v += BLOCK) {
            const u32x4 q = kv[v];
            count_key(h, q.x, lb, b);
            count_key(h, q.y, lb, b);
            count_key(h, q.z, lb, b);
            count_key(h, q.w, lb, b);
        }
        for (uint64_t k = (v1 << 2) + threadIdx.x; k < k1; k += BLOCK) count_key(h, keys[k], lb, b);
    }
    __syncthreads();
    uint32_t *row = part + ((uint64_t)s << bits) + ((uint64_t)b << lb);
    for (uint32_t i = threadIdx.x; i < (1u << lb); i += BLOCK) row[i] = h[i];
}

__global__ void __launch_bounds__(256) keyhist_reduce_kernel(const uint32_t *__restrict__ part, uint32_t S,
                                                            uint32_t bits, uint32_t *__restrict__ hist) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= (1u << bits)) return;
    // S is a multiple of 8: eight independent loads in flight per step
    uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    for (uint32_t s = 0; s < S; s += 8) {
#pragma unroll
        for (uint32_t r = 0; r < 8; ++r) acc[r] += part[((uint64_t)(s + r) << bits) + i];
    }
    const uint32_t v = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    if (v) hist[i] += v;
}

}  // namespace

KeyhistShape keyhist_shape(uint64_t M, uint32_t bits) {
    KeyhistShape k;
    const uint32_t lb = std::min(bits, LDS_BITS);
    const uint32_t NB = 1u << (bits - lb);
    // about 512 workgroups (two rounds over 256 CUs at one 128 KiB workgroup
    // each), slabs of at least 64 Ki keys, partial rows of at most
    // KEYHIST_PART_BYTES
    uint64_t S = std::max<uint64_t>(8, (512 / NB) & ~7ull);
    S = std::min<uint64_t>(S, std::max<uint64_t>(8, (M >> 16) & ~7ull));
    S = std::min<uint64_t>(S, std::max<uint64_t>(8, (KEYHIST_PART_BYTES / ((uint64_t)4 << bits)) & ~7ull));
    k.S = (uint32_t)S;
    k.slab = ((M + S - 1) / S + 3) & ~3ull;
    k.part_bytes = (size_t)S * ((size_t)4 << bits);
    k.grid = (uint32_t)S * NB;
    return k;
}

hipError_t launch_keyhist(const uint32_t *keys, uint64_t M, uint32_t bits, uint32_t *part, uint32_t *hist,
                          hipStream_t s) {
    if (!M) return hipSuccess;
    if (bits > KEYHIST_MAX_BITS) return hipErrorInvalidValue;
    const KeyhistShape k = keyhist_shape(M, bits);
    hipLaunchKernelGGL(keyhist_kernel, dim3(k.grid), dim3(BLOCK), 0, s, keys, M, bits, k.slab, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(keyhist_reduce_kernel, dim3(((1u << bits) + 255) / 256), dim3(256), 0, s, part, k.S, bits,
                       hist);
    return hipGetLastError();
}

}  // namespace pbit
