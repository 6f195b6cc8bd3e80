// Gibbs sampling of Feynman paths on the p-bit lattice (gfx950).
//
// One Markov chain per lane.  The chain's lattice (W words) lives in VGPRs;
// its free bits are also kept packed (F, up to 8 words) so the current
// value of a free bit is one bit-field extract.  A sweep visits the colours
// of the free-bit conflict graph in order; inside a colour the bits are
// conditionally independent and are visited Philox block by Philox block
// (block j serves free bits 4j..4j+3).  Per block:
//   u_t = word t of Philox4x32-10(counter = (sweep, j, chain, cid), key = seed)
//                                                    -- Fig. 2 step 1
//   new_t = (u_t < T), T = 2^31 for uniform circuits, else the uint32
//         threshold read from the LDS-staged table at the bits of the
//         factor scope                               -- Fig. 2 step 2 (heat bath)
//   flips = (new ^ old) & (bits of this colour)
//   lattice ^= TOG[j][flips]: one LDS row that holds the XOR of the cones
//         of the flipped bits (all 16 subsets precomputed per block), so the
//         four updates of a block cost one gather instead of four divergent
//         cone toggles.  Bits of one colour never touch each other's factor
//         scopes, so computing the four thresholds before the toggle is
//         exact.
// After every binned sweep the lane evaluates its path's output state alpha
// (bits of the last layer) and phase bin (the phase polynomial: popcounts
// of lattice AND bit planes for linear terms, of lattice AND shifted
// lattice for quadratic terms) and adds one to hist[alpha 2^K + k]
// (Fig. 2 step 3), privatised in LDS when the histogram fits.
//
// The circuit image is a __restrict__ kernel argument read at wave-uniform
// addresses, so it is fetched with scalar loads.
#pragma once
#include <hip/hip_runtime.h>

#include "blob.h"
#include "gibbs.h"
#include "phase.h"
#include "philox.h"

namespace pbit {

// One workgroup's share of a launch: stage the circuit's tables in LDS, run
// local chains lc0 .. lc0 + blockDim.x - 1 of the circuit for the launch's
// sweeps, flush the private histogram.  Shared by the single-circuit kernel
// and the persistent batched kernel (batched.hip).
// dst[i] = src[i] for i < n by the whole workgroup, eight loads per thread
// issued before their stores
template <class T>
__device__ __forceinline__ void stage_lds(T *dst, const T *__restrict__ src, uint32_t n) {
    constexpr uint32_t U = 8;
    for (uint32_t i0 = threadIdx.x; i0 < n; i0 += U * blockDim.x) {
        T v[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * blockDim.x;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * blockDim.x;
            if (i < n) dst[i] = v[u];
        }
    }
}

template <int W, bool UNIFORM, bool TOG>
__device__ __forceinline__ void gibbs_block(const uint32_t *__restrict__ B, uint32_t *__restrict__ state,
                                            uint32_t *__restrict__ hist, const GibbsArgs &a, uint32_t lc0,
                                            uint32_t *lds) {
    constexpr int TW = (W + 3) & ~3;
    const uint32_t fw = B[H_FW];
    const uint32_t h = B[H_H];
    const uint32_t ncol = B[H_NCOL];
    const uint32_t K = B[H_K];
    const uint32_t n = B[H_N];
    const uint32_t cid = B[H_CID];
    const bool uniform = UNIFORM || B[H_UNIFORM] != 0u;
    const uint32_t tog_words = TOG ? B[H_NBLK] * 16u * TW : 0u;
    // threshold tables in LDS, or read from the image when too large
    const bool thr_glob = !uniform && B[H_THR_TOTAL] > THR_LDS_MAX_WORDS;
    const uint32_t thr_total = uniform || thr_glob ? 0u : B[H_THR_TOTAL];
    const uint32_t nbins = 1u << B[H_HBITS];
    const uint32_t nblk = B[H_NBLK];
    uint32_t *lds_tog = lds;
    uint32_t *lds_thr = lds + tog_words;
    uint32_t *lds_h = lds_thr + thr_total;
    const uint32_t tid = threadIdx.x;
    const uint32_t lc = lc0 + tid;
    const bool active = lc < a.n_chains;

    // staging: eight loads per thread in flight before their stores, so a
    // small workgroup does not wait one memory latency per piece
    if (TOG) stage_lds<uint4>(reinterpret_cast<uint4 *>(lds_tog), reinterpret_cast<const uint4 *>(B + B[H_OFF_TOG]),
                              tog_words / 4);
    if (!uniform) stage_lds<uint32_t>(lds_thr, B + B[H_OFF_THRTAB], thr_total);
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
            for (int w = 0; w < W; ++w) x[w] = (uint32_t)w < Wc ? state[(size_t)w * a.n_chains + lc] : 0u;
        } else {
            const uint32_t *cw = B + B[H_OFF_CONST];
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] = cw[w];
        }
        // packed free bits
        uint32_t F[MAX_FW];
#pragma unroll
        for (int k = 0; k < MAX_FW; ++k) F[k] = 0u;
        if (!UNIFORM && a.resume) {
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
            if (UNIFORM) {
                // Every conditional is 1/2, so a sweep redraws every free bit
                // independently of the lattice: the lattice after the sweep
                // is const ^ XOR_j TOG[j][new bits of block j], the same
                // words the per-update cone toggles produce.  The next
                // block's Philox runs while this block's row is read.
                const uint32_t *cw = B + B[H_OFF_CONST];
#pragma unroll
                for (int w = 0; w < W; ++w) x[w] = cw[w];
                U4 u = philox4x32_10(s, 0u, chain, ctag, a.seed_lo, a.seed_hi);
                for (uint32_t j = 0; j < nblk; ++j) {
                    // u < 2^31 <=> top bit clear; rows ignore bits >= h
                    const uint32_t nb =
                        ((u.x >> 31) | ((u.y >> 30) & 2u) | ((u.z >> 29) & 4u) | ((u.w >> 28) & 8u)) ^ 15u;
                    uint4 r[TW / 4];
                    const uint4 *row = reinterpret_cast<const uint4 *>(lds_tog + (j * 16u + nb) * TW);
#pragma unroll
                    for (int q = 0; q < TW / 4; ++q) r[q] = row[q];
                    if (j + 1u < nblk) u = philox4x32_10(s, j + 1u, chain, ctag, a.seed_lo, a.seed_hi);
#pragma unroll
                    for (int q = 0; q < TW / 4; ++q) {
                        if (4 * q + 0 < W) x[4 * q + 0] ^= r[q].x;
                        if (4 * q + 1 < W) x[4 * q + 1] ^= r[q].y;
                        if (4 * q + 2 < W) x[4 * q + 2] ^= r[q].z;
                        if (4 * q + 3 < W) x[4 * q + 3] ^= r[q].w;
                    }
                }
                // three-qubit permutation gates: each derived AND variable,
                // in layer order, read off the lattice so far
                const uint32_t ny = B[H_NY];
                const uint32_t *yr = B + B[H_OFF_Y];
                const uint32_t ys = y_stride(B[H_WS]);
                for (uint32_t j = 0; j < ny; ++j) {
                    const uint32_t p = yr[j * ys], q = yr[j * ys + 1];
                    const uint32_t y = (select_word<W>(x, p >> 5) >> (p & 31)) & (select_word<W>(x, q >> 5) >> (q & 31));
                    const uint32_t m = 0u - (y & 1u);
#pragma unroll
                    for (int w = 0; w < W; ++w) x[w] ^= m & yr[j * ys + 2 + w];
                }
            } else
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
                            uint32_t nb;
                            if (uniform) {
                                nb = ((u.x >> 31) | ((u.y >> 30) & 2u) | ((u.z >> 29) & 4u) | ((u.w >> 28) & 8u)) ^ 15u;
                            } else {
                                const uint32_t uu[4] = {u.x, u.y, u.z, u.w};
                                nb = 0u;
#pragma unroll
                                for (int t = 0; t < 4; ++t)
                                    if (m & (1u << t)) {
                                        const uint32_t T = threshold_of<W>(B, 4 * j + t, x, lds_thr, thr_glob);
                                        nb |= (uu[t] < T ? 1u : 0u) << t;
                                    }
                            }
                            const uint32_t sh = (4u * j) & 31u;
                            const uint32_t fl = (nb ^ (F[k] >> sh)) & m;
                            F[k] ^= fl << sh;
                            if (TOG) {
                                const uint4 *row = reinterpret_cast<const uint4 *>(lds_tog + (j * 16u + fl) * TW);
#pragma unroll
                                for (int q = 0; q < TW / 4; ++q) {
                                    const uint4 r = row[q];
                                    if (4 * q + 0 < W) x[4 * q + 0] ^= r.x;
                                    if (4 * q + 1 < W) x[4 * q + 1] ^= r.y;
                                    if (4 * q + 2 < W) x[4 * q + 2] ^= r.z;
                                    if (4 * q + 3 < W) x[4 * q + 3] ^= r.w;
                                }
                            } else {
#pragma unroll
                                for (int t = 0; t < 4; ++t) {
                                    const uint32_t *cm = cone + (4 * j + t) * W;
                                    if ((fl >> t) & 1u) {
#pragma unroll
                                        for (int w = 0; w < W; ++w) x[w] ^= cm[w];
                                    }
                                }
                            }
                        }
                    }
                }
            }
            if (s >= a.bin_from && !meets_soft_zero<W>(B, x)) {
                const uint32_t bin = phase_and_bin<W>(B, x, K, n);
                if (a.lds_hist)
                    atomicAdd(&lds_h[bin], 1u);
                else
                    atomicAdd(&hist[bin], 1u);
            }
        }
        if (state) {
#pragma unroll
            for (int w = 0; w < W; ++w)
                if ((uint32_t)w < Wc) state[(size_t)w * a.n_chains + lc] = x[w];
        }
    }
    if (a.lds_hist) {
        __syncthreads();
        for (uint32_t i = tid; i < nbins; i += blockDim.x) {
            const uint32_t v = lds_h[i];
            if (v) atomicAdd(&hist[i], v);
        }
    }
}

}  // namespace pbit
