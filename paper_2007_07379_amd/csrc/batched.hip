// Persistent batched Gibbs launch: many circuits of uneven n, d and chain
// counts in one launch per lattice-width class.  The host cuts every
// circuit's chains into tiles of one workgroup (256 chains), sorts the tiles
// by decreasing cost (free bits x lattice words, longest first), and the
// resident workgroups pull tiles from an atomic counter until the list is
// exhausted; each tile runs the same per-chain sweep body as the
// single-circuit kernel, so every chain's lattice and every count equals a
// separate run of that circuit bit for bit.
#include <hip/hip_runtime.h>

#include "batched.h"
#include "gibbs_body.h"

namespace pbit {

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    return (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)v) |
           ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32);
}

__global__ void reset_queue_kernel(uint32_t *q) {
    if (threadIdx.x == 0) *q = 0u;
}

// The tile index and everything read from the tile and circuit tables is
// the same for every lane: in scalar registers, and the circuit's pointers
// derived from the kernel's base pointers, so the image is read with scalar
// loads and the state and histogram with global (not generic) instructions.
template <int WMAX>
__global__ __launch_bounds__(256) void batched_kernel(BatchArgs a, const uint32_t *__restrict__ blob_base,
                                                      uint32_t *__restrict__ state_base,
                                                      uint32_t *__restrict__ hist_base) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ uint32_t slot;
    for (;;) {
        if (threadIdx.x == 0) slot = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t t = uniform_u32(slot);
        __syncthreads();  // every lane has read the slot before it is reused
        if (t >= a.ntiles) break;
        const BatchTile T = a.tiles[t];
        const BatchCirc C = a.circs[uniform_u32(T.circ)];
        const uint32_t *__restrict__ blob = blob_base + uniform_u64(C.blob_off);
        uint32_t *state = state_base ? state_base + uniform_u64(C.state_off) : nullptr;
        uint32_t *hist = hist_base + uniform_u64(C.hist_off);
        GibbsArgs g;
        g.n_chains = uniform_u32(C.n_chains);
        g.chain_begin = a.chain_begin;
        g.seed_lo = a.seed_lo;
        g.seed_hi = a.seed_hi;
        g.sweep_begin = a.sweep_begin;
        g.n_sweeps = a.n_sweeps;
        g.bin_from = a.bin_from;
        g.resume = a.resume;
        g.lds_hist = uniform_u32(C.lds_hist);
        switch (uniform_u32(C.Wk)) {
#define PBIT_CASE(V)                                                                     \
    case V:                                                                              \
        if (V <= WMAX)                                                                   \
            gibbs_block<(V <= WMAX ? V : 1), true, true>(blob, state, hist, g, uniform_u32(T.c0), lds);   \
        break;
            PBIT_CASE(1)
            PBIT_CASE(2)
            PBIT_CASE(3)
            PBIT_CASE(4)
            PBIT_CASE(6)
            PBIT_CASE(8)
            PBIT_CASE(10)
            PBIT_CASE(12)
            PBIT_CASE(13)
            PBIT_CASE(14)
            PBIT_CASE(16)
            PBIT_CASE(17)
            PBIT_CASE(20)
            PBIT_CASE(24)
            PBIT_CASE(28)
            PBIT_CASE(32)
#undef PBIT_CASE
            default:
                break;
        }
        __syncthreads();  // the LDS tables of the next tile may differ
    }
}

int batched_class_of(uint32_t Wk) { return Wk <= 8 ? 0 : (Wk <= 17 ? 1 : 2); }

hipError_t launch_batched(int cls, const BatchArgs &a, const uint32_t *blob_base, uint32_t *state_base,
                          uint32_t *hist_base, uint32_t grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, a.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void *fn = cls == 0 ? (const void *)batched_kernel<8>
                              : (cls == 1 ? (const void *)batched_kernel<17> : (const void *)batched_kernel<32>);
    if (lds > 65536) {
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (cls == 0)
        hipLaunchKernelGGL(batched_kernel<8>, dim3(grid), dim3(256), lds, s, a, blob_base, state_base, hist_base);
    else if (cls == 1)
        hipLaunchKernelGGL(batched_kernel<17>, dim3(grid), dim3(256), lds, s, a, blob_base, state_base, hist_base);
    else
        hipLaunchKernelGGL(batched_kernel<32>, dim3(grid), dim3(256), lds, s, a, blob_base, state_base, hist_base);
    return hipGetLastError();
}

}  // namespace pbit
