// Device helpers shared by the sampling kernels (internal): lattice word
// selection, LDS threshold lookup, and the phase polynomial / output state
// of a path (Eq. (path): the phase of a path is the sum of its gates' phase
// bins; Fig. 2 step 3: the sample is binned at its output state).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "blob.h"

namespace pbit {

template <int W>
__device__ __forceinline__ uint32_t select_word(const uint32_t (&x)[W + 2], uint32_t w) {
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < W; ++i)
        if ((uint32_t)i == w) r = x[i];
    return r;
}

// True if the lattice meets a soft zero of a gate (an entry replaced by
// e^(-J) for sampling): such a path is not one of the circuit's, and the
// sample is not binned.
template <int W>
__device__ __forceinline__ bool meets_soft_zero(const uint32_t *__restrict__ B, const uint32_t (&x)[W + 2]) {
    const uint32_t ns = B[H_NSOFT];
    const uint32_t *r = B + B[H_OFF_SOFT];
    for (uint32_t g = 0; g < ns; ++g, r += SOFT_STRIDE) {
        uint32_t idx = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t p = r[j];
            idx |= ((select_word<W>(x, p >> 5) >> (p & 31)) & 1u) << j;
        }
        if ((r[4] >> idx) & 1u) return true;
    }
    return false;
}

// Threshold of free bit b for the lattice x: from the tables staged in LDS
// (lds_thr), or from the image when they did not fit (thr_glob).  The two
// reads are separate so each is an LDS or a global load, not a generic one.
template <int W>
__device__ __forceinline__ uint32_t threshold_of(const uint32_t *__restrict__ B, uint32_t b,
                                                 const uint32_t (&x)[W + 2], const uint32_t *lds_thr,
                                                 bool thr_glob) {
    const uint32_t *rec = B + B[H_OFF_THRINFO] + b * THR_STRIDE;
    const uint32_t toff = rec[0], ns = rec[1];
    uint32_t idx = 0;
    for (uint32_t j = 0; j < ns; ++j) {
        const uint32_t p = rec[2 + j];
        const uint32_t v = select_word<W>(x, p >> 5);
        idx |= ((v >> (p & 31)) & 1u) << j;
    }
    if (thr_glob) return B[B[H_OFF_THRTAB] + toff + idx];
    // an LDS pointer by type, so the compiler keeps this an LDS read
    typedef const __attribute__((address_space(3))) uint32_t lds_u32;
    return ((lds_u32 *)lds_thr)[toff + idx];
}

template <int W>
__device__ __forceinline__ uint32_t phase_and_bin(const uint32_t *__restrict__ B, const uint32_t (&x)[W + 2],
                                                  uint32_t K, uint32_t n) {
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
            for (int w = 0; w < W; ++w) y[w] = x[w] & __builtin_amdgcn_alignbit(x[w + 2], x[w + 1], delta - 32);
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
    // merged groups: popcount(x & OR_delta(shift_delta(x) & mask_delta))
    const uint32_t nqg = B[H_NQG];
    const uint32_t *grec = B + B[H_OFF_QG];
    for (uint32_t g = 0; g < nqg; ++g) {
        const uint32_t t = grec[0];
        const uint32_t m = grec[1];
        grec += 2;
        uint32_t z[W];
#pragma unroll
        for (int w = 0; w < W; ++w) z[w] = 0u;
        for (uint32_t e = 0; e < m; ++e) {
            const uint32_t delta = grec[0];
            const uint32_t *mk = grec + 1;
            if (delta < 32) {
#pragma unroll
                for (int w = 0; w < W; ++w)
                    z[w] = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_alignbit(x[w + 1], x[w], delta), mk[w], z[w],
                                                       0xEA);  // (a & b) | c
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w)
                    z[w] = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_alignbit(x[w + 2], x[w + 1], delta - 32),
                                                       mk[w], z[w], 0xEA);
            }
            grec += 1 + W;
        }
        uint32_t cnt = 0u;
#pragma unroll
        for (int w = 0; w < W; ++w) cnt += __builtin_popcount(x[w] & z[w]);
#pragma unroll
        for (int tt = 0; tt < MAX_K; ++tt)
            if ((uint32_t)tt == t) acc[tt] += cnt;
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
    return (alpha << K) | ph;
}

}  // namespace pbit
