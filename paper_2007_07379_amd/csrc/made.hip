// MADE learned proposal on gfx950: bf16 MFMA GEMM with degree-mask tile
// skipping and fused epilogues, loss gradient, column sums, Adam with FP32
// master weights and bf16 shadows, log q of given paths, and the fused
// autoregressive sampler.
//
// Every matrix product (forward, backward, sampler) is a sequence of
// v_mfma_f32_16x16x32_bf16 accumulating 32-wide K chunks in ascending order
// from zero, never split.  Masked weights are exact zeros, so a chunk that
// lies beyond a unit's degree adds exact zeros: the fused sampler (which
// stops at the last chunk a unit needs) and the batched forward (which runs
// to the end of the tile's range) give the same bits for every logit, and
// log q of a sampled path equals the scorer's log q of that path.
#include <hip/hip_runtime.h>

#include <cmath>

#include "blob.h"
#include "made.h"
#include "made_kernels.h"
#include "philox.h"

namespace pbit {

typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 32, LDSK = TK + 8;

// ---------------------------------------------------------------------------
// GEMM
// ---------------------------------------------------------------------------
// Loads one 64 x 32 operand tile (rows r0.., k k0..) into LDS laid out
// [row][k] (k contiguous), zero outside [0, R) x [0, kend).
__device__ __forceinline__ void load_tile(bf16 (*T)[LDSK], const bf16 *src, int64_t sr, int64_t sk, int r0, int R,
                                          int k0, int kend) {
    const int t = threadIdx.x;
    if (sk == 1) {
        const int r = t >> 2, kk = (t & 3) * 8;
        const int gr = r0 + r, gk = k0 + kk;
        const bf16 *p = src + (int64_t)gr * sr + gk;
        if (gr < R && gk + 8 <= kend && (((uintptr_t)p) & 15) == 0) {
            *reinterpret_cast<bf16x8 *>(&T[r][kk]) = *reinterpret_cast<const bf16x8 *>(p);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) T[r][kk + i] = (gr < R && gk + i < kend) ? p[i] : (bf16)0.0f;
        }
    } else if (sr == 1) {
        const int k = t >> 3, rr = (t & 7) * 8;
        const int gk = k0 + k, gr = r0 + rr;
        const bf16 *p = src + (int64_t)gk * sk + gr;
        if (gk < kend && gr + 8 <= R && (((uintptr_t)p) & 15) == 0) {
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(p);
#pragma unroll
            for (int i = 0; i < 8; ++i) T[rr + i][k] = v[i];
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) T[rr + i][k] = (gk < kend && gr + i < R) ? p[i] : (bf16)0.0f;
        }
    } else {
        for (int e = t; e < TM * TK; e += 256) {
            const int r = e / TK, k = e % TK;
            const int gr = r0 + r, gk = k0 + k;
            T[r][k] = (gr < R && gk < kend) ? src[(int64_t)gr * sr + (int64_t)gk * sk] : (bf16)0.0f;
        }
    }
}

__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    __shared__ __align__(16) bf16 As[TM][LDSK];
    __shared__ __align__(16) bf16 Bs[TN][LDSK];
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int nt = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    int kb = g.kbeg ? g.kbeg[nt] : 0;
    int ke = g.kend ? g.kend[nt] : g.K;
    // a tile whose every output is masked needs no reduction
    bool dead = false;
    if (g.deg_row && g.deg_col) {
        const int mlast = min(m0 + TM, g.M) - 1, nlast = min(n0 + TN, g.N) - 1;
        dead = g.deg_row[m0] > g.deg_col[nlast];
        (void)mlast;
    }
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (!dead) {
        for (int k0 = 0; k0 < ke; k0 += TK) {
            if (k0 + TK <= kb) continue;  // chunks entirely below the range are zero
            load_tile(As, g.A, g.sam, g.sak, m0, g.M, k0, ke);
            load_tile(Bs, g.B, g.sbn, g.sbk, n0, g.N, k0, ke);
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&As[wr + i * 16 + (lane & 15)][(lane >> 4) * 8]);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Bs[wc + j * 16 + (lane & 15)][(lane >> 4) * 8]);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wr + i * 16 + (lane >> 4) * 4 + e;
                const int n = n0 + wc + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][e];
                if (g.bias) v += g.bias[n];
                if (g.relu) v = v > 0.f ? v : 0.f;
                if (g.gate && !((float)g.gate[(int64_t)m * g.sgm + (int64_t)n * g.sgn] > 0.f)) v = 0.f;
                if (g.deg_row && g.deg_col && g.deg_row[m] > g.deg_col[n]) v = 0.f;
                const int64_t o = (int64_t)m * g.scm + (int64_t)n * g.scn;
                if (g.out_bf16)
                    reinterpret_cast<bf16 *>(g.C)[o] = (bf16)v;
                else if (g.accumulate)
                    reinterpret_cast<float *>(g.C)[o] += v;
                else
                    reinterpret_cast<float *>(g.C)[o] = v;
            }
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
    dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// element-wise helpers
// ---------------------------------------------------------------------------
// Lattice words (word-major, word w of sample b at states[w n + b]) -> bf16
// 0/1 rows X[b][i], zero for i >= D.
__global__ void unpack_kernel(const uint32_t *__restrict__ states, int n, int D, int DP, bf16 *__restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * DP) return;
    const int b = (int)(e / DP), i = (int)(e % DP);
    float v = 0.f;
    if (i < D) v = (float)((states[(int64_t)(i >> 5) * n + b] >> (i & 31)) & 1u);
    X[e] = (bf16)v;
}

// dLoss/dL = (sigmoid(L) - x) / n on free positions; the batch-mean binary
// cross-entropy is accumulated into *loss.
__global__ void loss_grad_kernel(const float *__restrict__ L, const bf16 *__restrict__ X, const int *__restrict__ freem,
                                 int n, int D, int DP, float inv_n, bf16 *__restrict__ G, float *__restrict__ loss) {
    __shared__ float red[256];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float nll = 0.f;
    if (e < (int64_t)n * D) {
        const int b = (int)(e / D), i = (int)(e % D);
        const float z = L[e];
        const float x = (float)X[(int64_t)b * DP + i];
        float gval = 0.f;
        if (freem[i]) {
            const float s = 1.f / (1.f + expf(-z));
            gval = (s - x) * inv_n;
            // softplus(-z) for x = 1, softplus(z) for x = 0
            const float zz = x > 0.5f ? -z : z;
            nll = (zz > 0.f ? zz + log1pf(expf(-zz)) : log1pf(expf(zz))) * inv_n;
        }
        G[e] = (bf16)gval;
    }
    red[threadIdx.x] = nll;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0]);
}

// Column sums of a row-major n x N bf16 matrix in two deterministic passes:
// workgroup (column tile, row chunk) sums its 256 rows for 64 columns (four
// row groups of 64 rows, combined in a fixed order), then each column adds
// its chunk partials in ascending chunk order.
__global__ __launch_bounds__(256) void colsum_part_kernel(const bf16 *__restrict__ G, int n, int N,
                                                          float *__restrict__ part) {
    __shared__ float red[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + tx;
    const int r0 = blockIdx.y * 256 + ty * 64;
    float s = 0.f;
    if (j < N) {
        const int r1 = min(r0 + 64, n);
        for (int b = r0; b < r1; ++b) s += (float)G[(int64_t)b * N + j];
    }
    red[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && j < N) part[(int64_t)blockIdx.y * N + j] = ((red[0][tx] + red[1][tx]) + red[2][tx]) + red[3][tx];
}

__global__ void colsum_final_kernel(const float *__restrict__ part, int chunks, int N, float *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * N + j];
    out[j] = s;
}

__global__ void adam_kernel(float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int64_t P, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] = th[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// bf16 shadows of one K x N weight (row-major) and its transpose N x KP
// (row n holds the K inputs of unit n, zero-padded to KP).
__global__ void shadow_kernel(const float *__restrict__ W, int K, int N, int KP, bf16 *__restrict__ Wb,
                              bf16 *__restrict__ WT) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * KP) return;
    const int n = (int)(e / KP), k = (int)(e % KP);
    const float w = k < K ? W[(int64_t)k * N + n] : 0.f;
    WT[e] = (bf16)w;
    if (k < K) Wb[(int64_t)k * N + n] = (bf16)w;
}

// ---------------------------------------------------------------------------
// log q of given paths (score mode)
// ---------------------------------------------------------------------------
__global__ void logq_kernel(const float *__restrict__ L, const uint32_t *__restrict__ states, uint64_t stride,
                            uint64_t b0, const int *__restrict__ fpos, int h, int n, int D, double *__restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    double s = 0.0;
    for (int f = 0; f < h; ++f) {
        const int p = fpos[f];
        const uint32_t x = (states[(uint64_t)(p >> 5) * stride + b0 + b] >> (p & 31)) & 1u;
        const uint32_t T = made_threshold(L[(int64_t)b * D + p]);
        s += made_log_prob(T, x);
    }
    out[b] = s;
}

// ---------------------------------------------------------------------------
// fused autoregressive sampler
// ---------------------------------------------------------------------------
// One wave samples 16 paths.  Free bits are visited in ascending lattice
// order; before free bit b (lattice position p) the hidden units whose
// degree became <= p are computed from the LDS-resident inputs, then the
// logit of position p, then the bit is drawn with Philox (tag 1) against the
// uint32 threshold of sigmoid(logit), log q accumulates log(T/2^32) or
// log(1 - T/2^32), and a set bit flips its cone in the inputs and in the
// lattice words, so the deterministic positions after p are always set.
// One chain of 16-row MFMA accumulations over nk 32-wide K chunks, in
// ascending order from chunk 0 into one accumulator (the order the batched
// GEMM uses, so every logit is the same bits).  The operands of up to eight
// chunks are loaded before their products, so a phase waits for one round
// of loads instead of one per chunk.
__device__ __forceinline__ f32x4 mfma_chunks(const bf16 *__restrict__ arow, const bf16 *__restrict__ brow, int nk) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    constexpr int G = 8;
    int c = 0;
    for (; c + G <= nk; c += G) {
        bf16x8 av[G], bv[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            av[g] = *reinterpret_cast<const bf16x8 *>(arow + (c + g) * 32);
            bv[g] = *reinterpret_cast<const bf16x8 *>(brow + (c + g) * 32);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[g], bv[g], acc, 0, 0, 0);
    }
    if (c < nk) {
        const int r = nk - c;  // 1..G-1 chunks left
        bf16x8 av[G], bv[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g < r) {
                av[g] = *reinterpret_cast<const bf16x8 *>(arow + (c + g) * 32);
                bv[g] = *reinterpret_cast<const bf16x8 *>(brow + (c + g) * 32);
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (g < r) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[g], bv[g], acc, 0, 0, 0);
    }
    return acc;
}

__global__ __launch_bounds__(64) void made_sample_kernel(SampleArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int CS = 16;
    const int DP = a.DP, H = a.H, W = a.W;
    bf16 *Xs = reinterpret_cast<bf16 *>(smem);           // [CS][DP]
    bf16 *H1s = Xs + CS * DP;                             // [CS][H]
    bf16 *H2s = H1s + CS * H;                             // [CS][H]
    float *logit = reinterpret_cast<float *>(H2s + CS * H);  // [CS]
    uint32_t *lat = reinterpret_cast<uint32_t *>(logit + CS);  // [CS][W]
    const int lane = threadIdx.x;
    const int c0 = blockIdx.x * CS;
    const uint32_t *B = a.blob;
    const uint32_t *cw = B + B[H_OFF_CONST];
    const uint32_t *cone = B + B[H_OFF_CONE];
    const uint32_t WS = B[H_WS];
    const uint32_t cid = B[H_CID];

    for (int e = lane; e < CS * DP; e += 64) {
        const int i = e % DP;
        Xs[e] = (bf16)((i < a.D) ? (float)((cw[i >> 5] >> (i & 31)) & 1u) : 0.f);
    }
    for (int e = lane; e < 2 * CS * H; e += 64) H1s[e] = (bf16)0.f;
    for (int e = lane; e < CS * W; e += 64) lat[e] = cw[e % W];
    __syncthreads();
    double lq = 0.0;
    const int row = lane & 15, kq = (lane >> 4) * 8;
    for (int f = 0; f < a.h; ++f) {
        const int4 ph = a.phase[f];  // {u1a, u1b, u2a, u2b}
        const int4 kk = a.phase_k[f];  // {K1 end, K2 end, K3 end, position p}
        const int p = kk.w;
        // (a) first-layer units whose degree became <= p
        for (int u0 = ph.x; u0 < ph.y; u0 += 16) {
            const int u = min(u0 + row, H - 1);
            const f32x4 acc = mfma_chunks(Xs + row * DP + kq, a.W1T + (int64_t)u * DP + kq, (kk.x + 31) / 32);
            const int un = u0 + row;
            if (un < ph.y) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = acc[e] + a.b1[un];
                    v = v > 0.f ? v : 0.f;
                    H1s[((lane >> 4) * 4 + e) * H + un] = (bf16)v;
                }
            }
        }
        __syncthreads();
        // (b) second-layer units whose degree became <= p
        for (int u0 = ph.z; u0 < ph.w; u0 += 16) {
            const int u = min(u0 + row, H - 1);
            const f32x4 acc = mfma_chunks(H1s + row * H + kq, a.W2T + (int64_t)u * H + kq, (kk.y + 31) / 32);
            const int un = u0 + row;
            if (un < ph.w) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = acc[e] + a.b2[un];
                    v = v > 0.f ? v : 0.f;
                    H2s[((lane >> 4) * 4 + e) * H + un] = (bf16)v;
                }
            }
        }
        __syncthreads();
        // (c) logit of position p (every column of the tile computes it)
        {
            const f32x4 acc = mfma_chunks(H2s + row * H + kq, a.VT + (int64_t)p * H + kq, (kk.z + 31) / 32);
            if (row == 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e) logit[(lane >> 4) * 4 + e] = acc[e] + a.c[p];
            }
        }
        __syncthreads();
        // (d) draw the bit (or read it from the scored path), flip its cone
        if (lane < CS) {
            const int chain = c0 + lane;
            if (chain < a.n) {
                const uint32_t T = made_threshold(logit[lane]);
                uint32_t bit;
                if (a.score) {
                    bit = (a.score[(int64_t)(p >> 5) * a.n + chain] >> (p & 31)) & 1u;
                } else {
                    const U4 u4 = philox4x32_10(a.step, (uint32_t)f >> 2, a.chain_begin + chain, cid | (1u << 16),
                                                a.seed_lo, a.seed_hi);
                    const uint32_t uu[4] = {u4.x, u4.y, u4.z, u4.w};
                    bit = uu[f & 3] < T ? 1u : 0u;
                }
                lq += made_log_prob(T, bit);
                // the lattice bit at p is the free bit itself: flip its cone
                // when the drawn value differs from the current one
                const uint32_t cur = (lat[lane * W + (p >> 5)] >> (p & 31)) & 1u;
                if (bit != cur) {
                    const uint32_t *cm = cone + (int64_t)f * WS;
                    for (int w = 0; w < W; ++w) {
                        uint32_t mw = cm[w];
                        lat[lane * W + w] ^= mw;
                        while (mw) {
                            const int i = 32 * w + __builtin_ctz(mw);
                            mw &= mw - 1;
                            const float xv = (float)Xs[lane * DP + i];
                            Xs[lane * DP + i] = (bf16)(1.f - xv);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (lane < CS) {
        const int chain = c0 + lane;
        if (chain < a.n) {
            if (a.out)
                for (int w = 0; w < W; ++w) a.out[(int64_t)w * a.n + chain] = lat[lane * W + w];
            a.logq[chain] = lq;
        }
    }
}

hipError_t launch_made_sample(const SampleArgs &a, hipStream_t s) {
    const int grid = (a.n + 15) / 16;
    const size_t lds = (size_t)16 * a.DP * 2 + (size_t)2 * 16 * a.H * 2 + 16 * 4 + (size_t)16 * a.W * 4;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)made_sample_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(made_sample_kernel, dim3(grid), dim3(64), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_unpack(const uint32_t *states, int n, int D, int DP, bf16 *X, hipStream_t s) {
    const int64_t tot = (int64_t)n * DP;
    hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, states, n, D, DP, X);
    return hipGetLastError();
}

hipError_t launch_loss_grad(const float *L, const bf16 *X, const int *freem, int n, int D, int DP, bf16 *G,
                            float *loss, hipStream_t s) {
    const int64_t tot = (int64_t)n * D;
    hipLaunchKernelGGL(loss_grad_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, L, X, freem, n, D, DP,
                       1.f / (float)n, G, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const bf16 *G, int n, int N, float *part, float *out, hipStream_t s) {
    const int chunks = (n + 255) / 256;
    if (chunks == 0 || N == 0) return hipSuccess;
    hipLaunchKernelGGL(colsum_part_kernel, dim3((N + 63) / 64, chunks), dim3(256), 0, s, G, n, N, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_final_kernel, dim3((N + 255) / 256), dim3(256), 0, s, part, chunks, N, out);
    return hipGetLastError();
}

hipError_t launch_adam(float *th, float *m, float *v, const float *g, int64_t P, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, th, m, v, g, P, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_shadow(const float *W, int K, int N, int KP, bf16 *Wb, bf16 *WT, hipStream_t s) {
    const int64_t tot = (int64_t)N * KP;
    hipLaunchKernelGGL(shadow_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, W, K, N, KP, Wb, WT);
    return hipGetLastError();
}

hipError_t launch_logq(const float *L, const uint32_t *states, uint64_t stride, uint64_t b0, const int *fpos, int h,
                       int n, int D, double *out, hipStream_t s) {
    hipLaunchKernelGGL(logq_kernel, dim3((n + 255) / 256), dim3(256), 0, s, L, states, stride, b0, fpos, h, n, D, out);
    return hipGetLastError();
}

}  // namespace pbit
