// Two lanes per chain: Gibbs sweeps of circuits whose conditionals are all
// 1/2, for runs with too few chains to give each SIMD two waves (65,536
// chains fill 1024 SIMDs with one wave each, so every stall of a single
// instruction stream is exposed).
//
// Lanes 2c and 2c+1 hold chain c; lane h (h = lane & 1) owns lattice words
// [h WH, h WH + WH), WH = ceil(W / 2).  Per pair of Philox blocks (2i, 2i+1)
// lane h computes block 2i + h, the two new-bit nibbles are swapped with
// one DPP move, and each lane XORs its half of both toggle rows.  The
// sample's phase is split the same way (each lane popcounts its own words;
// the two partial sums and the two halves of the output state meet in one
// DPP move each), and the even lane adds the count.  Every lattice word and
// count equals the one-lane kernel's.
#include <hip/hip_runtime.h>

#include "blob.h"
#include "gibbs.h"
#include "philox.h"

namespace pbit {

__device__ __forceinline__ uint32_t pair_swap(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
}

// LDS layout of the pair kernel:
//   toggle rows  [(j * 16 + f) * 2 + half][WHP]
//   phase masks  [entry * 2 + half][WHP]; entries: K linear planes, then
//                K planes of every per-offset record, then the mask of
//                every merged-group member (in blob order)
//   histogram    [2^(n+K)] when privatised
template <int W>
__global__ __launch_bounds__(512) void gibbs_pair_kernel(const uint32_t *__restrict__ B, uint32_t *__restrict__ state,
                                                         uint32_t *__restrict__ hist, GibbsArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];
    constexpr int WH = (W + 1) / 2;
    constexpr int WHP = (WH + 3) & ~3;
    const uint32_t K = B[H_K];
    const uint32_t n = B[H_N];
    const uint32_t cid = B[H_CID];
    const uint32_t nblk = B[H_NBLK];
    const uint32_t TW = B[H_TOGW];
    const uint32_t nqd = B[H_NQD];
    const uint32_t nqg = B[H_NQG];
    const uint32_t nbins = 1u << B[H_HBITS];
    const uint32_t tid = threadIdx.x;
    const uint32_t half = tid & 1u;

    // count phase-mask entries
    uint32_t nent = K + nqd * K;
    {
        const uint32_t *g = B + B[H_OFF_QG];
        for (uint32_t q = 0; q < nqg; ++q) {
            const uint32_t m = g[1];
            nent += m;
            g += 2 + m * (1 + W);
        }
    }
    const uint32_t tog_words = nblk * 16u * 2u * WHP;
    const uint32_t msk_words = nent * 2u * WHP;
    uint32_t *lds_tog = lds;
    uint32_t *lds_msk = lds + tog_words;
    uint32_t *lds_h = lds_msk + msk_words;

    // stage toggle rows, split by half
    {
        const uint32_t *tog = B + B[H_OFF_TOG];
        for (uint32_t e = tid; e < tog_words; e += blockDim.x) {
            const uint32_t i = e % WHP, hh = (e / WHP) & 1u, row = e / (2u * WHP);
            const uint32_t w = hh * WH + i;
            lds_tog[e] = (i < (uint32_t)WH && w < (uint32_t)W) ? tog[row * TW + w] : 0u;
        }
    }
    // stage phase masks, split by half
    for (uint32_t e = tid; e < msk_words; e += blockDim.x) {
        const uint32_t i = e % WHP, hh = (e / WHP) & 1u, ent = e / (2u * WHP);
        const uint32_t w = hh * WH + i;
        uint32_t v = 0u;
        if (i < (uint32_t)WH && w < (uint32_t)W) {
            if (ent < K) {
                v = B[B[H_OFF_LIN] + ent * W + w];
            } else if (ent < K + nqd * K) {
                const uint32_t r = (ent - K) / K, t = (ent - K) % K;
                v = B[B[H_OFF_QD] + r * (2 + K * W) + 2 + t * W + w];
            } else {
                uint32_t left = ent - K - nqd * K;
                const uint32_t *g = B + B[H_OFF_QG];
                for (uint32_t q = 0; q < nqg; ++q) {
                    const uint32_t m = g[1];
                    if (left < m) {
                        v = g[2 + left * (1 + W) + 1 + w];
                        break;
                    }
                    left -= m;
                    g += 2 + m * (1 + W);
                }
            }
        }
        lds_msk[e] = v;
    }
    if (a.lds_hist)
        for (uint32_t i = tid; i < nbins; i += blockDim.x) lds_h[i] = 0u;
    __syncthreads();

    const uint32_t lc = (blockIdx.x * blockDim.x + tid) >> 1;
    const bool active = lc < a.n_chains;
    if (active) {
        const uint32_t Wc = B[H_W];
        uint32_t x[WH + 2];
        uint32_t cw[WH];
        {
            const uint32_t *c = B + B[H_OFF_CONST];
#pragma unroll
            for (int i = 0; i < WH; ++i) {
                const uint32_t w0 = i, w1 = WH + i;
                const uint32_t v0 = c[w0], v1 = w1 < (uint32_t)W ? c[w1] : 0u;
                cw[i] = half ? v1 : v0;
            }
        }
#pragma unroll
        for (int i = 0; i < WH; ++i) {
            const uint32_t w = half * WH + i;
            x[i] = a.resume ? ((w < Wc) ? state[(size_t)w * a.n_chains + lc] : 0u) : cw[i];
        }
        x[WH] = x[WH + 1] = 0u;
        const uint32_t chain = a.chain_begin + lc;
        const uint32_t ctag = cid;
        const uint32_t linmask = B[H_LINMASK];
        const uint32_t aw = B[H_AWORD], ash = B[H_ASHIFT];

        for (uint32_t it = 0; it < a.n_sweeps; ++it) {
            const uint32_t s = a.sweep_begin + it;
#pragma unroll
            for (int i = 0; i < WH; ++i) x[i] = cw[i];
            uint32_t jm = half;
            U4 u = philox4x32_10(s, jm, chain, ctag, a.seed_lo, a.seed_hi);
            for (uint32_t j0 = 0; j0 < nblk; j0 += 2) {
                uint32_t nb = ((u.x >> 31) | ((u.y >> 30) & 2u) | ((u.z >> 29) & 4u) | ((u.w >> 28) & 8u)) ^ 15u;
                if (j0 + half >= nblk) nb = 0u;
                const uint32_t nbo = pair_swap(nb);
                const uint32_t ne = half ? nbo : nb, no = half ? nb : nbo;
                uint4 re[WHP / 4], ro[WHP / 4];
                const uint4 *rowe = reinterpret_cast<const uint4 *>(lds_tog + ((j0 * 16u + ne) * 2u + half) * WHP);
#pragma unroll
                for (int q = 0; q < WHP / 4; ++q) re[q] = rowe[q];
                const bool has_odd = j0 + 1u < nblk;
                if (has_odd) {
                    const uint4 *rowo =
                        reinterpret_cast<const uint4 *>(lds_tog + (((j0 + 1u) * 16u + no) * 2u + half) * WHP);
#pragma unroll
                    for (int q = 0; q < WHP / 4; ++q) ro[q] = rowo[q];
                }
                jm = j0 + 2u + half;
                if (j0 + 2u < nblk) u = philox4x32_10(s, jm, chain, ctag, a.seed_lo, a.seed_hi);
#pragma unroll
                for (int q = 0; q < WHP / 4; ++q) {
                    if (4 * q + 0 < WH) x[4 * q + 0] ^= re[q].x;
                    if (4 * q + 1 < WH) x[4 * q + 1] ^= re[q].y;
                    if (4 * q + 2 < WH) x[4 * q + 2] ^= re[q].z;
                    if (4 * q + 3 < WH) x[4 * q + 3] ^= re[q].w;
                }
                if (has_odd) {
#pragma unroll
                    for (int q = 0; q < WHP / 4; ++q) {
                        if (4 * q + 0 < WH) x[4 * q + 0] ^= ro[q].x;
                        if (4 * q + 1 < WH) x[4 * q + 1] ^= ro[q].y;
                        if (4 * q + 2 < WH) x[4 * q + 2] ^= ro[q].z;
                        if (4 * q + 3 < WH) x[4 * q + 3] ^= ro[q].w;
                    }
                }
            }
            if (s >= a.bin_from) {
                // the even lane needs the odd lane's first two words for the
                // funnel shifts; the odd lane's words past W are zero
                const uint32_t e0 = pair_swap(x[0]), e1 = pair_swap(WH > 1 ? x[1] : 0u);
                x[WH] = half ? 0u : e0;
                x[WH + 1] = half ? 0u : (WH > 1 ? e1 : 0u);
                uint32_t acc = 0u;
                uint32_t ent = 0;
#pragma unroll
                for (int t = 0; t < MAX_K; ++t) {
                    if ((uint32_t)t < K) {
                        if ((linmask >> t) & 1u) {
                            const uint4 *mk = reinterpret_cast<const uint4 *>(lds_msk + (ent * 2u + half) * WHP);
                            uint32_t cnt = 0u;
#pragma unroll
                            for (int q = 0; q < WHP / 4; ++q) {
                                const uint4 m4 = mk[q];
                                if (4 * q + 0 < WH) cnt += __builtin_popcount(x[4 * q + 0] & m4.x);
                                if (4 * q + 1 < WH) cnt += __builtin_popcount(x[4 * q + 1] & m4.y);
                                if (4 * q + 2 < WH) cnt += __builtin_popcount(x[4 * q + 2] & m4.z);
                                if (4 * q + 3 < WH) cnt += __builtin_popcount(x[4 * q + 3] & m4.w);
                            }
                            acc += cnt << t;
                        }
                        ++ent;
                    }
                }
                const uint32_t *qrec = B + B[H_OFF_QD];
                for (uint32_t r = 0; r < nqd; ++r) {
                    const uint32_t delta = qrec[0], pm = qrec[1];
                    uint32_t y[WH];
#pragma unroll
                    for (int i = 0; i < WH; ++i)
                        y[i] = x[i] & (delta < 32 ? __builtin_amdgcn_alignbit(x[i + 1], x[i], delta)
                                                  : __builtin_amdgcn_alignbit(x[i + 2], x[i + 1], delta - 32));
                    for (uint32_t t = 0; t < K; ++t) {
                        if ((pm >> t) & 1u) {
                            const uint4 *mk = reinterpret_cast<const uint4 *>(lds_msk + (ent * 2u + half) * WHP);
                            uint32_t cnt = 0u;
#pragma unroll
                            for (int q = 0; q < WHP / 4; ++q) {
                                const uint4 m4 = mk[q];
                                if (4 * q + 0 < WH) cnt += __builtin_popcount(y[4 * q + 0] & m4.x);
                                if (4 * q + 1 < WH) cnt += __builtin_popcount(y[4 * q + 1] & m4.y);
                                if (4 * q + 2 < WH) cnt += __builtin_popcount(y[4 * q + 2] & m4.z);
                                if (4 * q + 3 < WH) cnt += __builtin_popcount(y[4 * q + 3] & m4.w);
                            }
                            acc += cnt << t;
                        }
                        ++ent;
                    }
                    qrec += 2 + K * W;
                }
                const uint32_t *grec = B + B[H_OFF_QG];
                for (uint32_t g = 0; g < nqg; ++g) {
                    const uint32_t t = grec[0], m = grec[1];
                    uint32_t z[WH];
#pragma unroll
                    for (int i = 0; i < WH; ++i) z[i] = 0u;
                    for (uint32_t e = 0; e < m; ++e) {
                        const uint32_t delta = grec[2 + e * (1 + W)];
                        const uint4 *mk = reinterpret_cast<const uint4 *>(lds_msk + (ent * 2u + half) * WHP);
                        uint32_t mw[WHP];
#pragma unroll
                        for (int q = 0; q < WHP / 4; ++q) {
                            const uint4 m4 = mk[q];
                            mw[4 * q] = m4.x;
                            mw[4 * q + 1] = m4.y;
                            mw[4 * q + 2] = m4.z;
                            mw[4 * q + 3] = m4.w;
                        }
                        if (delta < 32) {
#pragma unroll
                            for (int i = 0; i < WH; ++i)
                                z[i] = __builtin_amdgcn_bitop3_b32(__builtin_amdgcn_alignbit(x[i + 1], x[i], delta),
                                                                   mw[i], z[i], 0xEA);
                        } else {
#pragma unroll
                            for (int i = 0; i < WH; ++i)
                                z[i] = __builtin_amdgcn_bitop3_b32(
                                    __builtin_amdgcn_alignbit(x[i + 2], x[i + 1], delta - 32), mw[i], z[i], 0xEA);
                        }
                        ++ent;
                    }
                    uint32_t cnt = 0u;
#pragma unroll
                    for (int i = 0; i < WH; ++i) cnt += __builtin_popcount(x[i] & z[i]);
                    acc += cnt << t;
                    grec += 2 + m * (1 + W);
                }
                acc += pair_swap(acc);
                const uint32_t ph = (acc + B[H_PCONST]) & ((1u << K) - 1u);
                // output state: words aw and aw + 1, each from its owner lane
                uint32_t lo = 0u, hi = 0u;
#pragma unroll
                for (int i = 0; i < WH; ++i) {
                    const uint32_t w = half * WH + i;
                    if (w == aw) lo = x[i];
                    if (w == aw + 1) hi = x[i];
                }
                lo |= pair_swap(lo);
                hi |= pair_swap(hi);
                const uint32_t alpha = __builtin_amdgcn_alignbit(hi, lo, ash) & ((1u << n) - 1u);
                const uint32_t bin = (alpha << K) | ph;
                if (!half) {
                    if (a.lds_hist)
                        atomicAdd(&lds_h[bin], 1u);
                    else
                        atomicAdd(&hist[bin], 1u);
                }
            }
        }
        if (state) {
#pragma unroll
            for (int i = 0; i < WH; ++i) {
                const uint32_t w = half * WH + i;
                if (w < Wc) state[(size_t)w * a.n_chains + lc] = x[i];
            }
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

size_t gibbs_pair_lds_bytes(const uint32_t *hb, bool lds_hist) {
    const uint32_t W = hb[H_WS];
    const uint32_t WH = (W + 1) / 2, WHP = (WH + 3) & ~3u;
    const uint32_t K = hb[H_K];
    uint32_t nent = K + hb[H_NQD] * K;
    const uint32_t *g = hb + hb[H_OFF_QG];
    for (uint32_t q = 0; q < hb[H_NQG]; ++q) {
        nent += g[1];
        g += 2 + g[1] * (1 + W);
    }
    size_t words = (size_t)hb[H_NBLK] * 16 * 2 * WHP + (size_t)nent * 2 * WHP;
    if (lds_hist) words += (size_t)1 << hb[H_HBITS];
    return words * sizeof(uint32_t);
}

#define PBIT_FOR_EACH_W(X) X(1) X(2) X(3) X(4) X(6) X(8) X(10) X(12) X(13) X(14) X(16) X(17) X(20) X(24) X(28) X(32)

hipError_t launch_gibbs_pair(uint32_t Wk, const GibbsLaunch &a, uint32_t block, size_t lds, hipStream_t stream) {
    const uint32_t grid = (2u * a.n_chains + block - 1) / block;
    if (grid == 0) return hipSuccess;
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
#define PBIT_LAUNCH(V)                                                                                       \
    if (Wk == V) {                                                                                           \
        if (lds > 65536) {                                                                                   \
            hipError_t e = hipFuncSetAttribute((const void *)gibbs_pair_kernel<V>,                           \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);        \
            if (e != hipSuccess) return e;                                                                   \
        }                                                                                                    \
        hipLaunchKernelGGL((gibbs_pair_kernel<V>), dim3(grid), dim3(block), lds, stream, a.blob, a.state,    \
                           a.hist, g);                                                                       \
        return hipGetLastError();                                                                            \
    }
    PBIT_FOR_EACH_W(PBIT_LAUNCH)
#undef PBIT_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace pbit
