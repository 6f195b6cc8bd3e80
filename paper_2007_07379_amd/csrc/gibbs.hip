// Gibbs sampling of Feynman paths on the p-bit lattice (gfx950).
//
// One Markov chain per lane.  The chain's lattice (W words) lives in VGPRs;
// its free bits are also kept packed (F, up to 8 words) so the current
// value of a free bit is one bit-field extract.  A sweep visits the colours
// of the free-bit conflict graph in order; inside a colour the bits are
// conditionally independent and are visited Philox block by Philox block
// (block j serves free bits 4j..4j+3).  Each update:
//   u  = word (b % 4) of Philox4x32-10(counter = (sweep, b/4, chain, cid),
//        key = seed)                               -- Fig. 2 step 1
//   T  = 2^31 for uniform circuits, else the uint32 threshold read from the
//        LDS-staged table at the bits of the factor scope
//   new = (u < T); if new != old: flip the bit's cone in the lattice
//                                                  -- Fig. 2 step 2 (heat bath)
// After every binned sweep the lane evaluates its path's output state alpha
// (bits of the last layer) and phase bin (the phase polynomial: popcounts
// of lattice AND bit planes for linear terms, of lattice AND shifted
// lattice for quadratic terms) and adds one to hist[alpha 2^K + k]
// (Fig. 2 step 3), privatised in LDS when the histogram fits.
//
// The circuit image is read with wave-uniform addresses (scalar loads).
#include <hip/hip_runtime.h>

#include "blob.h"
#include "gibbs.h"
#include "philox.h"

namespace pbit {

template <int W>
__device__ __forceinline__ uint32_t select_word(const uint32_t (&x)[W + 2], uint32_t w) {
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < W; ++i)
        if ((uint32_t)i == w) r = x[i];
    return r;
}

template <int W>
__device__ __forceinline__ uint32_t threshold_of(const uint32_t *__restrict__ B, uint32_t b,
                                                 const uint32_t (&x)[W + 2], const uint32_t *lds_thr) {
    const uint32_t *rec = B + B[H_OFF_THRINFO] + b * THR_STRIDE;
    const uint32_t toff = rec[0], ns = rec[1];
    uint32_t idx = 0;
    for (uint32_t j = 0; j < ns; ++j) {
        const uint32_t p = rec[2 + j];
        const uint32_t v = select_word<W>(x, p >> 5);
        idx |= ((v >> (p & 31)) & 1u) << j;
    }
    return lds_thr[toff + idx];
}

template <int W, bool UNIFORM>
__global__ __launch_bounds__(256) void gibbs_kernel(GibbsLaunch a) {
    extern __shared__ uint32_t lds[];
    const uint32_t *__restrict__ B = a.blob;
    const uint32_t h = B[H_H];
    const uint32_t fw = B[H_FW];
    const uint32_t ncol = B[H_NCOL];
    const uint32_t K = B[H_K];
    const uint32_t n = B[H_N];
    const uint32_t cid = B[H_CID];
    const uint32_t thr_total = UNIFORM ? 0u : B[H_THR_TOTAL];
    const uint32_t nbins = 1u << B[H_HBITS];
    uint32_t *lds_thr = lds;
    uint32_t *lds_h = lds + thr_total;
    const uint32_t tid = threadIdx.x;
    const uint32_t lc = blockIdx.x * blockDim.x + tid;
    const bool active = lc < a.n_chains;

    if (!UNIFORM) {
        const uint32_t *tab = B + B[H_OFF_THRTAB];
        for (uint32_t i = tid; i < thr_total; i += blockDim.x) lds_thr[i] = tab[i];
    }
    if (a.lds_hist)
        for (uint32_t i = tid; i < nbins; i += blockDim.x) lds_h[i] = 0u;
    __syncthreads();

    if (active) {
        uint32_t x[W + 2];
        x[W] = 0u;
        x[W + 1] = 0u;
        const uint32_t Wc = B[H_W];  // words stored per chain (<= W)
        if (a.resume) {
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] = (uint32_t)w < Wc ? a.state[(size_t)w * a.n_chains + lc] : 0u;
        } else {
            const uint32_t *cw = B + B[H_OFF_CONST];
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] = cw[w];
        }
        // packed free bits
        uint32_t F[MAX_FW];
#pragma unroll
        for (int k = 0; k < MAX_FW; ++k) F[k] = 0u;
        if (a.resume) {
            const uint32_t *fpos = B + B[H_OFF_FPOS];
            for (uint32_t b = 0; b < h; ++b) {
                const uint32_t p = fpos[b];
                const uint32_t bit = (select_word<W>(x, p >> 5) >> (p & 31)) & 1u;
#pragma unroll
                for (int k = 0; k < MAX_FW; ++k)
                    if ((uint32_t)k == (b >> 5)) F[k] |= bit << (b & 31);
            }
        }
        const uint32_t chain = a.chain_begin + lc;
        const uint32_t *colidx = B + B[H_OFF_COLIDX];
        const uint32_t *colent = B + B[H_OFF_COLENT];
        const uint32_t *cone = B + B[H_OFF_CONE];
        const uint32_t ctag = cid;  // tag 0: Gibbs updates

        for (uint32_t it = 0; it < a.n_sweeps; ++it) {
            const uint32_t s = a.sweep_begin + it;
            for (uint32_t c = 0; c < ncol; ++c) {
#pragma unroll
                for (int k = 0; k < MAX_FW; ++k) {
                    if ((uint32_t)k < fw) {
                        const uint32_t off = colidx[(c * MAX_FW + k) * 2];
                        const uint32_t cnt = colidx[(c * MAX_FW + k) * 2 + 1];
                        for (uint32_t e = 0; e < cnt; ++e) {
                            const uint32_t ent = colent[off + e];
                            const uint32_t j = ent >> 4;
                            const uint32_t m = ent & 15u;
                            const U4 u = philox4x32_10(s, j, chain, ctag, a.seed_lo, a.seed_hi);
                            const uint32_t uu[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                if (m & (1u << t)) {
                                    const uint32_t b = 4 * j + t;
                                    const uint32_t bp = b & 31u;
                                    const uint32_t T = UNIFORM ? 0x80000000u : threshold_of<W>(B, b, x, lds_thr);
                                    const uint32_t nb = uu[t] < T ? 1u : 0u;
                                    const uint32_t ob = (F[k] >> bp) & 1u;
                                    if (nb != ob) {
                                        F[k] ^= 1u << bp;
                                        const uint32_t *cm = cone + b * W;
#pragma unroll
                                        for (int w = 0; w < W; ++w) x[w] ^= cm[w];
                                    }
                                }
                            }
                        }
                    }
                }
            }
            if (s >= a.bin_from) {
                // phase polynomial
                uint32_t acc[MAX_K];
#pragma unroll
                for (int t = 0; t < MAX_K; ++t) acc[t] = 0u;
                const uint32_t linmask = B[H_LINMASK];
                const uint32_t *lin = B + B[H_OFF_LIN];
#pragma unroll
                for (int t = 0; t < MAX_K; ++t) {
                    if ((uint32_t)t < K && ((linmask >> t) & 1u)) {
#pragma unroll
                        for (int w = 0; w < W; ++w) acc[t] += __builtin_popcount(x[w] & lin[t * W + w]);
                    }
                }
                const uint32_t nqd = B[H_NQD];
                const uint32_t *qrec = B + B[H_OFF_QD];
                const uint32_t qstride = 2 + K * W;
                for (uint32_t q = 0; q < nqd; ++q) {
                    const uint32_t delta = qrec[0];
                    const uint32_t pm = qrec[1];
                    uint32_t y[W];
                    if (delta < 32) {
#pragma unroll
                        for (int w = 0; w < W; ++w) y[w] = x[w] & __builtin_amdgcn_alignbit(x[w + 1], x[w], delta);
                    } else {
#pragma unroll
                        for (int w = 0; w < W; ++w)
                            y[w] = x[w] & __builtin_amdgcn_alignbit(x[w + 2], x[w + 1], delta - 32);
                    }
#pragma unroll
                    for (int t = 0; t < MAX_K; ++t) {
                        if ((uint32_t)t < K && ((pm >> t) & 1u)) {
#pragma unroll
                            for (int w = 0; w < W; ++w) acc[t] += __builtin_popcount(y[w] & qrec[2 + t * W + w]);
                        }
                    }
                    qrec += qstride;
                }
                uint32_t ph = B[H_PCONST];
#pragma unroll
                for (int t = 0; t < MAX_K; ++t) ph += acc[t] << t;
                ph &= (1u << K) - 1u;
                // output state: lattice bits [d n, d n + n)
                const uint32_t aw = B[H_AWORD], ash = B[H_ASHIFT];
                uint32_t lo = 0u, hi = 0u;
#pragma unroll
                for (int w = 0; w < W; ++w)
                    if ((uint32_t)w == aw) {
                        lo = x[w];
                        hi = x[w + 1];
                    }
                const uint32_t alpha = __builtin_amdgcn_alignbit(hi, lo, ash) & ((1u << n) - 1u);
                const uint32_t bin = (alpha << K) | ph;
                if (a.lds_hist)
                    atomicAdd(&lds_h[bin], 1u);
                else
                    atomicAdd(&a.hist[bin], 1u);
            }
        }
        if (a.state) {
#pragma unroll
            for (int w = 0; w < W; ++w)
                if ((uint32_t)w < Wc) a.state[(size_t)w * a.n_chains + lc] = x[w];
        }
    }
    if (a.lds_hist) {
        __syncthreads();
        for (uint32_t i = tid; i < nbins; i += blockDim.x) {
            const uint32_t v = lds_h[i];
            if (v) atomicAdd(&a.hist[i], v);
        }
    }
}

// the widths of KERNEL_WIDTHS (blob.h)
#define PBIT_FOR_EACH_W(X) X(1) X(2) X(3) X(4) X(6) X(8) X(10) X(12) X(13) X(14) X(16) X(17) X(20) X(24) X(28) X(32)

hipError_t launch_gibbs(uint32_t Wk, bool uniform, const GibbsLaunch &a, uint32_t block, size_t lds_bytes,
                        hipStream_t stream) {
    const uint32_t grid = (a.n_chains + block - 1) / block;
    if (grid == 0) return hipSuccess;
#define PBIT_LAUNCH(V)                                                                                    \
    if (Wk == V) {                                                                                        \
        const void *fn = uniform ? (const void *)gibbs_kernel<V, true> : (const void *)gibbs_kernel<V, false>; \
        if (lds_bytes > 65536) {                                                                          \
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes); \
            if (e != hipSuccess) return e;                                                                \
        }                                                                                                 \
        if (uniform)                                                                                      \
            hipLaunchKernelGGL((gibbs_kernel<V, true>), dim3(grid), dim3(block), lds_bytes, stream, a);  \
        else                                                                                              \
            hipLaunchKernelGGL((gibbs_kernel<V, false>), dim3(grid), dim3(block), lds_bytes, stream, a); \
        return hipGetLastError();                                                                         \
    }
    PBIT_FOR_EACH_W(PBIT_LAUNCH)
#undef PBIT_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace pbit
