// Single-circuit Gibbs sampling kernel and its launcher (gfx950); the
// per-chain sweep body is in gibbs_body.h.
#include <hip/hip_runtime.h>

#include "blob.h"
#include "gibbs.h"
#include "gibbs_body.h"

namespace pbit {

template <int W, bool UNIFORM, bool TOG>
__global__ __launch_bounds__(256) void gibbs_kernel(const uint32_t *__restrict__ B, uint32_t *__restrict__ state,
                                                    uint32_t *__restrict__ hist, GibbsArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];
    gibbs_block<W, UNIFORM, TOG>(B, state, hist, a, blockIdx.x * blockDim.x, lds);
}

size_t gibbs_lds_bytes(const uint32_t *hb, bool tog, bool lds_hist) {
    const uint32_t WS = hb[H_WS];
    const uint32_t TW = (WS + 3) & ~3u;
    size_t words = 0;
    if (tog) words += (size_t)hb[H_NBLK] * 16 * TW;
    words += hb[H_UNIFORM] || hb[H_THR_TOTAL] > THR_LDS_MAX_WORDS ? 0 : hb[H_THR_TOTAL];
    if (lds_hist) words += (size_t)1 << hb[H_HBITS];
    return words * sizeof(uint32_t);
}

// the widths of KERNEL_WIDTHS (blob.h)
#define PBIT_FOR_EACH_W(X) X(1) X(2) X(3) X(4) X(6) X(8) X(10) X(12) X(13) X(14) X(16) X(17) X(20) X(24) X(28) X(32)

template <int V, bool U, bool T>
static hipError_t launch_one(const GibbsLaunch &a, uint32_t grid, uint32_t block, size_t lds, hipStream_t stream) {
    const void *fn = (const void *)gibbs_kernel<V, U, T>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    GibbsArgs g;
    g.n_chains = a.n_chains;
    g.chain_begin = a.chain_begin;
    g.seed_lo = a.seed_lo;
    g.seed_hi = a.seed_hi;
    g.sweep_begin = a.sweep_begin;
    g.n_sweeps = a.n_sweeps;
    g.bin_from = a.bin_from;
    g.resume = a.resume;
    g.lds_hist = a.lds_hist;
    hipLaunchKernelGGL((gibbs_kernel<V, U, T>), dim3(grid), dim3(block), lds, stream, a.blob, a.state, a.hist, g);
    return hipGetLastError();
}

hipError_t launch_gibbs(uint32_t Wk, bool uniform, bool tog, const GibbsLaunch &a, uint32_t block, size_t lds_bytes,
                        hipStream_t stream) {
    const uint32_t grid = (a.n_chains + block - 1) / block;
    if (grid == 0) return hipSuccess;
#define PBIT_LAUNCH(V)                                                                           \
    if (Wk == V) {                                                                               \
        if (tog && uniform) return launch_one<V, true, true>(a, grid, block, lds_bytes, stream); \
        if (tog) return launch_one<V, false, true>(a, grid, block, lds_bytes, stream);           \
        return launch_one<V, false, false>(a, grid, block, lds_bytes, stream);                   \
    }
    PBIT_FOR_EACH_W(PBIT_LAUNCH)
#undef PBIT_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace pbit
