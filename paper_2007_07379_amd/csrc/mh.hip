// Metropolis-Hastings accept of independence proposals (Fig. 2 step 2 with
// the acceptance ratio on |exp(-E)|, i.e. on exp(-Re E) only):
//   log r = [ln|psi(x')| - ln|psi(x)|] + [log q(x) - log q(x')],
//   accept iff u < min(1, exp(log r)) 2^32, u = Philox4x32-10 word 0 at
//   counter (step, 0, chain, circuit_id | 2 << 16).
// ln|psi| = sum of ln|U_g| over the gates with non-constant magnitude (the
// others add the same constant to every path); for circuits without such
// gates the first bracket is exactly zero.  The post-transition path is
// binned (Fig. 2 step 3): one sample per transition.
#include <hip/hip_runtime.h>

#include "blob.h"
#include "made_kernels.h"
#include "phase.h"
#include "philox.h"

namespace pbit {

// ln|psi| of two paths x and y at once: the sum, in gate order, of ln|U_g|
// over the real-energy records (`rec`, nre records of RE_STRIDE words; the
// tables are read with a per-lane index, so the caller passes a copy in LDS
// when it has one)
template <int W>
__device__ __forceinline__ void log_weights(const uint32_t *rec, uint32_t nre, const uint32_t (&x)[W + 2],
                                            const uint32_t (&y)[W + 2], double &sx, double &sy) {
    sx = 0.0;
    sy = 0.0;
    for (uint32_t r = 0; r < nre; ++r, rec += RE_STRIDE) {
        const uint32_t a = rec[0];
        uint32_t ix = 0, ox = 0, iy = 0, oy = 0;
        for (uint32_t j = 0; j < a; ++j) {
            const uint32_t pi = rec[1 + j], po = rec[3 + j];
            ix |= ((select_word<W>(x, pi >> 5) >> (pi & 31)) & 1u) << j;
            ox |= ((select_word<W>(x, po >> 5) >> (po & 31)) & 1u) << j;
            iy |= ((select_word<W>(y, pi >> 5) >> (pi & 31)) & 1u) << j;
            oy |= ((select_word<W>(y, po >> 5) >> (po & 31)) & 1u) << j;
        }
        const uint32_t tx = ox * (1u << a) + ix, ty = oy * (1u << a) + iy;
        sx += __longlong_as_double((long long)((uint64_t)rec[8 + 2 * tx] | ((uint64_t)rec[9 + 2 * tx] << 32)));
        sy += __longlong_as_double((long long)((uint64_t)rec[8 + 2 * ty] | ((uint64_t)rec[9 + 2 * ty] << 32)));
    }
}

// real-energy records staged in LDS when they take at most this many words
constexpr uint32_t MH_LDS_RE_WORDS = 8192;

// Histograms of at most this many bins are privatised in LDS per workgroup
// (every chain adds one count per transition, and circuits with few output
// states would otherwise serialise on a handful of HBM addresses).
constexpr uint32_t MH_LDS_BINS = 8192;

// One chain's accept; returns the bin of its post-transition path, or -1
// when it has none to add (no histogram, or no chain for this thread).
template <int W>
__device__ __forceinline__ int mh_accept_body(const MhArgs &a, const uint32_t *re) {
    const uint32_t *__restrict__ B = a.blob;
    const int lc = blockIdx.x * blockDim.x + threadIdx.x;
    if (lc >= a.n) return -1;
    const uint32_t Wc = B[H_W];
    uint32_t x[W + 2], y[W + 2];
    x[W] = x[W + 1] = y[W] = y[W + 1] = 0u;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        x[w] = (uint32_t)w < Wc ? a.state[(int64_t)w * a.n + lc] : 0u;
        y[w] = (uint32_t)w < Wc ? a.prop[(int64_t)w * a.n + lc] : 0u;
    }
    double lr = a.logq_cur[lc] - a.logq_prop[lc];
    if (B[H_NRE]) {
        double wx, wy;
        log_weights<W>(re, B[H_NRE], x, y, wx, wy);
        lr += wy - wx;
    }
    const double acc = lr >= 0.0 ? 1.0 : exp(lr);
    const uint32_t cid = B[H_CID];
    const U4 u = philox4x32_10(a.step, 0u, a.chain_begin + (uint32_t)lc, cid | (2u << 16), a.seed_lo, a.seed_hi);
    const bool accept = (double)u.x < acc * 4294967296.0;
    if (accept) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            x[w] = y[w];
            if ((uint32_t)w < Wc) a.state[(int64_t)w * a.n + lc] = y[w];
        }
    }
    if (a.accepts && accept) a.accepts[lc] += 1ull;
    return a.hist ? (int)phase_and_bin<W>(B, x, B[H_K], B[H_N]) : -1;
}

template <int W>
__global__ __launch_bounds__(256) void mh_accept_kernel(MhArgs a) {
    extern __shared__ uint32_t lds_h[];
    const bool priv = a.hist && a.hist_bins <= MH_LDS_BINS;
    // LDS: the privatised histogram, then the real-energy records
    const uint32_t nre_w = a.blob[H_NRE] * (uint32_t)RE_STRIDE;
    const bool re_lds = nre_w <= MH_LDS_RE_WORDS;
    uint32_t *re_s = lds_h + (priv ? a.hist_bins : 0u);
    if (re_lds) {
        const uint32_t *re_g = a.blob + a.blob[H_OFF_RE];
        for (uint32_t i = threadIdx.x; i < nre_w; i += blockDim.x) re_s[i] = re_g[i];
    }
    if (priv)
        for (uint32_t i = threadIdx.x; i < a.hist_bins; i += blockDim.x) lds_h[i] = 0u;
    __syncthreads();
    // separate calls, so the records' and the histogram's address spaces are
    // known to the compiler (LDS reads and atomics, not generic ones)
    const int bin = re_lds ? mh_accept_body<W>(a, re_s) : mh_accept_body<W>(a, a.blob + a.blob[H_OFF_RE]);
    if (bin >= 0) {
        if (priv)
            atomicAdd(&lds_h[bin], 1u);
        else
            atomicAdd(&a.hist[bin], 1u);
    }
    if (priv) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < a.hist_bins; i += blockDim.x) {
            const uint32_t v = lds_h[i];
            if (v) atomicAdd(&a.hist[i], v);
        }
    }
}

// Per-path observables of chain states (Eq. (path)): the bin alpha 2^K + phi
// of each path and ln|psi| over the gates with non-constant magnitude (the
// real-energy records; the other gates add one constant to every path).
template <int W>
__global__ __launch_bounds__(256) void observe_kernel(const uint32_t *__restrict__ B, const uint32_t *state, int n,
                                                     uint32_t *bin, double *logmag) {
    const int lc = blockIdx.x * blockDim.x + threadIdx.x;
    if (lc >= n) return;
    const uint32_t Wc = B[H_W];
    uint32_t x[W + 2];
    x[W] = x[W + 1] = 0u;
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = (uint32_t)w < Wc ? state[(int64_t)w * n + lc] : 0u;
    if (bin) bin[lc] = phase_and_bin<W>(B, x, B[H_K], B[H_N]);
    if (logmag) {
        double s = 0.0, unused = 0.0;
        if (B[H_NRE]) log_weights<W>(B + B[H_OFF_RE], B[H_NRE], x, x, s, unused);
        logmag[lc] = s;
    }
}

#define PBIT_FOR_EACH_W(X) X(1) X(2) X(3) X(4) X(6) X(8) X(10) X(12) X(13) X(14) X(16) X(17) X(20) X(24) X(28) X(32)

hipError_t launch_observe(uint32_t Wk, const uint32_t *blob, const uint32_t *state, int n, uint32_t *bin,
                          double *logmag, hipStream_t s) {
    const int grid = (n + 255) / 256;
    if (grid == 0) return hipSuccess;
#define PBIT_LAUNCH(V)                                                                               \
    if (Wk == V) {                                                                                   \
        hipLaunchKernelGGL((observe_kernel<V>), dim3(grid), dim3(256), 0, s, blob, state, n, bin, logmag); \
        return hipGetLastError();                                                                    \
    }
    PBIT_FOR_EACH_W(PBIT_LAUNCH)
#undef PBIT_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_mh_accept(uint32_t Wk, const MhArgs &a, hipStream_t s) {
    const int grid = (a.n + 255) / 256;
    if (grid == 0) return hipSuccess;
    size_t lds = (a.hist && a.hist_bins <= MH_LDS_BINS) ? (size_t)a.hist_bins * 4 : 0;
    // the records are staged when they fit (the kernel reads their count from
    // the image; the launch reserves the largest staged size)
    lds += (size_t)MH_LDS_RE_WORDS * 4;
#define PBIT_LAUNCH(V)                                                                  \
    if (Wk == V) {                                                                      \
        hipLaunchKernelGGL((mh_accept_kernel<V>), dim3(grid), dim3(256), lds, s, a);    \
        return hipGetLastError();                                                       \
    }
    PBIT_FOR_EACH_W(PBIT_LAUNCH)
#undef PBIT_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace pbit
