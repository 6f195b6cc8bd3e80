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

#include <algorithm>
#include <cmath>
#include <cstring>

#include "blob.h"
#include "made.h"
#include "made_kernels.h"
#include "philox.h"

namespace pbit {

typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Workgroup tile TT x TT, TT = 64 (four waves of 32 x 32, each 2 x 2 MFMA
// tiles of 16 x 16).  K advances in stages of two 32-wide chunks staged
// through double-buffered LDS; the global loads of a stage are issued P
// stages ahead into registers, so their latency hides behind the products
// of the stages in between.  The 64 tile gives a product four workgroups per
// CU (36 KiB of LDS each), which the small products of training need to
// hide latency, and each tile has its own 64-column K range.  Prefetch
// depth, measured at 1, 2, 3 and 6 stages: 1 and 2 tie, 3 is 5 % slower, 6
// a quarter slower.
constexpr int TK = 32, TKS = 2 * TK, LDSK = TKS + 8;
constexpr int GEMM_P = 2;

// Operands are addressed as X(r, k) = src[r sr + k sk]; everything outside
// [0, R) x [0, kend) reads as zero.
//   Mode 0 (sk == 1, sr a multiple of 8, 16-byte aligned base): each 16-byte
//     load is 8 consecutive k of one row.
//   Mode 1 (sr == 1, sk a multiple of 8, aligned base): loads come in pairs,
//     rows k and k + 1 of 8 consecutive r, written to LDS as (k, k + 1)
//     pairs per r.
//   Mode 2: any other layout, element by element.
// Modes 0 and 1 never branch per load: a stage that is not interior to the
// operand loads from a clamped address and masks by dword, so every stage
// issues the same loads and their latency overlaps with earlier stages.
typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));

struct StageRegs {
    u32x4v v[4];
    int rem[4];     // valid elements of each segment (masked at the LDS store,
    bool interior;  // so no load waits before the stage is stored)
};

// LDS row layout: the eight 16-byte units of a row (8 k each) are stored in
// the order u ^ ((row >> 3) & 7).  Rows 8 apart fall on the same banks (a row
// pitch is a multiple of 16 bytes), and the pair stores of mode 1 write rows
// 8 apart from neighbouring lanes; the swizzle spreads them over eight units.
__device__ __forceinline__ int lds_col(int row, int k) { return (((k >> 3) ^ ((row >> 3) & 7)) << 3) | (k & 7); }

// dword d of a 16-byte segment holds elements 2d, 2d + 1; rem valid elements
__device__ __forceinline__ u32x4v seg_mask(int rem) {
    u32x4v m;
#pragma unroll
    for (int d = 0; d < 4; ++d) m[d] = rem >= 2 * d + 2 ? 0xFFFFFFFFu : (rem == 2 * d + 1 ? 0x0000FFFFu : 0u);
    return m;
}

// ROWS rows x TKS k per stage: ROWS / 32 segments of 8 elements per thread
template <int MODE, int ROWS>
__device__ __forceinline__ void stage_load(StageRegs &st, const bf16 *__restrict__ src, int64_t sr, int64_t sk, int r0,
                                           int R, int k0, int kend) {
    const int t = threadIdx.x;
    constexpr int NS = ROWS / 32, RB = ROWS / 8;
    if (MODE == 0) {
        st.interior = r0 + ROWS <= R && k0 + TKS <= kend;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int seg = t + 256 * j;  // ROWS rows x 8 segments of 8
            const int r = seg >> 3, kk = (seg & 7) * 8;
            const int gr = r0 + r, gk = k0 + kk;
            const int rem = st.interior ? 8 : (gr < R ? kend - gk : 0);
            const bf16 *p = rem > 0 ? src + (int64_t)gr * sr + gk : src;
            st.v[j] = *reinterpret_cast<const u32x4v *>(p);
            st.rem[j] = rem;
        }
    } else if (MODE == 1) {
        st.interior = r0 + ROWS <= R && k0 + TKS <= kend;
#pragma unroll
        for (int b = 0; b < NS / 2; ++b) {
            const int blk = t + 256 * b;  // RB row blocks of 8 x 32 k pairs
            const int rb = (blk % RB) * 8, kp = (blk / RB) * 2;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int gk = k0 + kp + j, gr = r0 + rb;
                const int rem = st.interior ? 8 : (gk < kend ? R - gr : 0);
                const bf16 *p = rem > 0 ? src + (int64_t)gk * sk + gr : src;
                st.v[2 * b + j] = *reinterpret_cast<const u32x4v *>(p);
                st.rem[2 * b + j] = rem;
            }
        }
    } else {
        st.interior = true;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int seg = t + 256 * j;
            const int r = seg >> 3, kk = (seg & 7) * 8;
            const int gr = r0 + r, gk = k0 + kk;
            bf16x8 e;
#pragma unroll
            for (int i = 0; i < 8; ++i)
                e[i] = (gr < R && gk + i < kend) ? src[(int64_t)gr * sr + (int64_t)(gk + i) * sk] : (bf16)0.0f;
            st.v[j] = __builtin_bit_cast(u32x4v, e);
        }
    }
}

template <int MODE, int ROWS>
__device__ __forceinline__ void stage_store(const StageRegs &st, bf16 (*T)[LDSK], bool kperm) {
    const int t = threadIdx.x;
    constexpr int NS = ROWS / 32, RB = ROWS / 8;
    u32x4v v[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) v[j] = st.interior ? st.v[j] : st.v[j] & seg_mask(st.rem[j]);
    if (MODE != 1 && kperm) {
        // the segment's two 4-unit pieces w, w + 1 of their 32-wide chunk go
        // to k-slots 8 (w & 3) + 4 (w >> 2)
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int seg = t + 256 * j, r = seg >> 3, kk = (seg & 7) * 8;
            const int base = kk & 32, w = (kk & 31) >> 2;
#pragma unroll
            for (int hpc = 0; hpc < 2; ++hpc) {
                const int wp = w + hpc, slot = base + 8 * (wp & 3) + 4 * (wp >> 2);
                *reinterpret_cast<uint2 *>(&T[r][lds_col(r, slot)]) = uint2{v[j][2 * hpc], v[j][2 * hpc + 1]};
            }
        }
    } else if (MODE != 1) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int seg = t + 256 * j, r = seg >> 3;
            *reinterpret_cast<u32x4v *>(&T[r][lds_col(r, (seg & 7) * 8)]) = v[j];
        }
    } else {
#pragma unroll
        for (int b = 0; b < NS / 2; ++b) {
            const int blk = t + 256 * b;
            const int rb = (blk % RB) * 8, kp = (blk / RB) * 2;
            const u32x4v a = v[2 * b], c = v[2 * b + 1];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // rows rb + 2q and rb + 2q + 1: (k, k + 1) pairs
                const int r = rb + 2 * q;
                *reinterpret_cast<uint32_t *>(&T[r][lds_col(r, kp)]) = (a[q] & 0xFFFFu) | (c[q] << 16);
                *reinterpret_cast<uint32_t *>(&T[r + 1][lds_col(r + 1, kp)]) = (a[q] >> 16) | (c[q] & 0xFFFF0000u);
            }
        }
    }
}

// One workgroup's tile (block bx of the tile order, split-K slice bz).
template <int MA, int MB, int TT>
__device__ __forceinline__ void gemm_body(const GemmArgs &g, int bx, int bz) {
    constexpr int TM = TT, TN = TT, F = TT / 32;  // F x F MFMA tiles per wave
    constexpr int P = GEMM_P;
    __shared__ __align__(16) bf16 As[2][TM][LDSK];
    __shared__ __align__(16) bf16 Bs[2][TN][LDSK];
    // XCD-aware tile order: workgroups are dispatched round-robin over the 8
    // XCDs (each with its own L2), so workgroup w runs on XCD w % 8; give each
    // XCD a contiguous run of row-major tiles, i.e. a band of row tiles that
    // share their A rows in that XCD's L2
    const int tn = (g.N + TN - 1) / TN, tm = (g.M + TM - 1) / TM;
    const int T = tn * tm, per = (T + 7) / 8;
    const int tile = (bx % 8) * per + bx / 8;
    if (tile >= T) return;
    const int tile_m = tile / tn, tile_n = tile % tn;
    const int m0 = tile_m * TM, n0 = tile_n * TN;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * (TT / 2), wc = (wave & 1) * (TT / 2);
    static_assert(TT == 64, "the K ranges kbeg / kend are per 64-column tile");
    // K range of the tile
    int kb = 0, ke = g.K;
    if (g.kbeg) kb = g.kbeg[tile_n];
    if (g.kend) ke = g.kend[tile_n];
    int c_lo = kb / TK, c_hi = (ke + TK - 1) / TK;  // 32-wide chunks [c_lo, c_hi)
    // split-K: slice bz of the chunk range
    if (g.ksplit > 1) {
        const int nc = c_hi - c_lo, per = (nc + g.ksplit - 1) / g.ksplit;
        c_lo = c_lo + bz * per;
        c_hi = min(c_hi, c_lo + per);
    }
    // a tile whose every output is masked needs no reduction
    if (g.deg_row && g.deg_col) {
        const int nlast = min(n0 + TN, g.N) - 1;
        if (g.deg_row[m0] > g.deg_col[nlast]) c_hi = c_lo;
    }
    f32x4 acc[F][F];
#pragma unroll
    for (int i = 0; i < F; ++i)
#pragma unroll
        for (int j = 0; j < F; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int S = c_hi > c_lo ? (c_hi - c_lo + 1) / 2 : 0;  // stages of two chunks
    if (S > 0) {
        // the stage's K end: the tile's, never past the slice
        const int kst = min(ke, c_hi * TK);
        StageRegs ra[P], rb[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            if (i < S) {
                stage_load<MA, TM>(ra[i], g.A, g.sam, g.sak, m0, g.M, (c_lo + 2 * i) * TK, kst);
                stage_load<MB, TN>(rb[i], g.B, g.sbn, g.sbk, n0, g.N, (c_lo + 2 * i) * TK, kst);
            }
        }
        stage_store<MA, TM>(ra[0], As[0], g.kperm);
        stage_store<MB, TN>(rb[0], Bs[0], g.kperm);
        __syncthreads();
        for (int sb = 0; sb < S; sb += P) {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const int st = sb + i;
                if (st < S) {
                    const int buf = st & 1;
                    // the registers of stage st went to LDS last iteration:
                    // reuse them for stage st + P
                    if (st + P < S) {
                        stage_load<MA, TM>(ra[i], g.A, g.sam, g.sak, m0, g.M, (c_lo + 2 * (st + P)) * TK, kst);
                        stage_load<MB, TN>(rb[i], g.B, g.sbn, g.sbk, n0, g.N, (c_lo + 2 * (st + P)) * TK, kst);
                    }
#pragma unroll
                    for (int kk = 0; kk < 2; ++kk) {
                        if (c_lo + 2 * st + kk < c_hi) {
                            bf16x8 af[F], bfr[F];
#pragma unroll
                            for (int a = 0; a < F; ++a) {
                                const int r = wr + a * 16 + (lane & 15);
                                af[a] = *reinterpret_cast<const bf16x8 *>(
                                    &As[buf][r][lds_col(r, kk * TK + (lane >> 4) * 8)]);
                            }
#pragma unroll
                            for (int b = 0; b < F; ++b) {
                                const int r = wc + b * 16 + (lane & 15);
                                bfr[b] = *reinterpret_cast<const bf16x8 *>(
                                    &Bs[buf][r][lds_col(r, kk * TK + (lane >> 4) * 8)]);
                            }
#pragma unroll
                            for (int a = 0; a < F; ++a)
#pragma unroll
                                for (int b = 0; b < F; ++b)
                                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0,
                                                                                        0);
                        }
                    }
                    if (st + 1 < S) {
                        stage_store<MA, TM>(ra[(i + 1) % P], As[buf ^ 1], g.kperm);
                        stage_store<MB, TN>(rb[(i + 1) % P], Bs[buf ^ 1], g.kperm);
                    }
                    __syncthreads();
                }
            }
        }
    }
    if (g.ksplit > 1 || g.keep_parts) {
        // raw partial sums of this slice; the reduction applies the epilogue
        float *part = g.part + (int64_t)bz * g.M * g.N;
#pragma unroll
        for (int i = 0; i < F; ++i)
#pragma unroll
            for (int j = 0; j < F; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int m = m0 + wr + i * 16 + (lane >> 4) * 4 + e;
                    const int n = n0 + wc + j * 16 + (lane & 15);
                    if (m < g.M && n < g.N) part[(int64_t)m * g.N + n] = acc[i][j][e];
                }
        return;
    }
    // epilogue: every operand the epilogue reads is loaded first, without
    // branches (clamped addresses), so the loads overlap; only the stores
    // are guarded
    float bias_j[F];
    int dcol[F], lfree[F];
#pragma unroll
    for (int j = 0; j < F; ++j) {
        const int n = n0 + wc + j * 16 + (lane & 15);
        const int nc = n < g.N ? n : g.N - 1;
        bias_j[j] = g.bias ? g.bias[nc] : 0.f;
        dcol[j] = g.deg_col ? g.deg_col[nc] : 0;
        lfree[j] = g.lossx ? g.lossfree[nc] : 0;
    }
    float csum[F];  // this lane's share of its columns' tile sums
#pragma unroll
    for (int j = 0; j < F; ++j) csum[j] = 0.f;
    float nll = 0.f;
    int drow[F][4];
#pragma unroll
    for (int i = 0; i < F; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = m0 + wr + i * 16 + (lane >> 4) * 4 + e;
            drow[i][e] = g.deg_row ? g.deg_row[m < g.M ? m : g.M - 1] : 0;
        }
    const bool masked = g.deg_row && g.deg_col;
#pragma unroll
    for (int i = 0; i < F; ++i) {
        bf16 gv[F][4];
        if (g.gate) {
#pragma unroll
            for (int j = 0; j < F; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int m = m0 + wr + i * 16 + (lane >> 4) * 4 + e;
                    const int n = n0 + wc + j * 16 + (lane & 15);
                    const int mc = m < g.M ? m : g.M - 1, nc = n < g.N ? n : g.N - 1;
                    gv[j][e] = g.gate[(int64_t)mc * g.sgm + (int64_t)nc * g.sgn];
                }
        }
#pragma unroll
        for (int j = 0; j < F; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wr + i * 16 + (lane >> 4) * 4 + e;
                const int n = n0 + wc + j * 16 + (lane & 15);
                float v = acc[i][j][e] + bias_j[j];
                if (g.relu) v = v > 0.f ? v : 0.f;
                if (g.gate && !((float)gv[j][e] > 0.f)) v = 0.f;
                if (masked && drow[i][e] > dcol[j]) v = 0.f;
                const bool inside = m < g.M && n < g.N;
                if (g.lossx) {
                    // v is the logit z: one exponential t = e^-|z| gives
                    // sigmoid(z) (1 / (1 + t) for z >= 0, t / (1 + t)
                    // below) and the loss, softplus(-z) for x = 1 and
                    // softplus(z) for x = 0, softplus(y) = max(y, 0) + log1p(t)
                    float gval = 0.f;
                    if (inside && lfree[j]) {
                        const float x = (float)g.lossx[(int64_t)m * g.slx + n];
                        const float t = expf(-fabsf(v));
                        const float r = __builtin_amdgcn_rcpf(1.f + t);  // 1 + t in [1, 2]
                        const float sg = v >= 0.f ? r : t * r;
                        gval = (sg - x) * g.inv_n;
                        const float zz = x > 0.5f ? -v : v;
                        nll += (fmaxf(zz, 0.f) + log1pf(t)) * g.inv_n;
                    }
                    v = gval;
                }
                float stored = 0.f;
                if (inside) {
                    const int64_t o = (int64_t)m * g.scm + (int64_t)n * g.scn;
                    if (g.out_bf16) {
                        const bf16 b = (bf16)v;
                        reinterpret_cast<bf16 *>(g.C)[o] = b;
                        stored = (float)b;
                    } else if (g.accumulate) {
                        reinterpret_cast<float *>(g.C)[o] += v;
                    } else {
                        reinterpret_cast<float *>(g.C)[o] = v;
                        stored = v;
                    }
                }
                csum[j] += stored;
            }
    }
    if (g.colpart) {
        // column sums over the tile's 64 rows: the four lane groups of a wave
        // (a fixed butterfly), then rows 0..31 plus rows 32..63
        __shared__ float cred[64];
#pragma unroll
        for (int j = 0; j < F; ++j) {
            csum[j] += __shfl_xor(csum[j], 16);
            csum[j] += __shfl_xor(csum[j], 32);
        }
        if (wr != 0 && lane < 16) {
#pragma unroll
            for (int j = 0; j < F; ++j) cred[wc + j * 16 + lane] = csum[j];
        }
        __syncthreads();
        if (wr == 0 && lane < 16) {
#pragma unroll
            for (int j = 0; j < F; ++j) {
                const int n = n0 + wc + j * 16 + lane;
                if (n < g.N) g.colpart[(int64_t)tile_m * g.N + n] = csum[j] + cred[wc + j * 16 + lane];
            }
        }
    }
    if (g.lossx) {
        // the tile's loss share: a butterfly within each wave, then the
        // four waves in order
        __shared__ float lred[4];
        for (int o = 32; o > 0; o >>= 1) nll += __shfl_xor(nll, o);
        if (lane == 0) lred[wave] = nll;
        __syncthreads();
        if (threadIdx.x == 0) g.losspart[tile] = ((lred[0] + lred[1]) + lred[2]) + lred[3];
    }
}

template <int MA, int MB, int TT>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    gemm_body<MA, MB, TT>(g, (int)blockIdx.x, (int)blockIdx.z);
}

// Several products of one operand layout in one launch: problem p takes
// blocks [start_p, start_p + nb_p), nb_p = bx_p z_p (bx_p, a multiple of 8,
// blocks of its tile order, z_p its slices), so the workgroups of all of them
// share the machine and one tail.  Block offsets stay multiples of 8, so a
// problem's tile order keeps its XCD mapping.
template <int MA, int MB>
__global__ __launch_bounds__(256) void gemm_group_kernel(GemmGroup gg) {
    int id = (int)blockIdx.x, p = 0;
    while (p + 1 < gg.count && id >= gg.bx[p] * gg.z[p]) {
        id -= gg.bx[p] * gg.z[p];
        ++p;
    }
    gemm_body<MA, MB, 64>(gg.g[p], id % gg.bx[p], id / gg.bx[p]);
}

// Split-K reduction: slices added in ascending order, degree mask, fp32 out.
// M N < 2^31 (checked at launch): 32-bit index arithmetic.
__global__ void splitk_reduce_kernel(GemmArgs g) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint32_t)g.M * (uint32_t)g.N) return;
    const int m = (int)(e / (uint32_t)g.N), n = (int)(e - (uint32_t)m * (uint32_t)g.N);
    float v = 0.f;
    for (int z = 0; z < g.ksplit; ++z) v += g.part[(int64_t)z * g.M * g.N + e];
    if (g.deg_row && g.deg_col && g.deg_row[m] > g.deg_col[n]) v = 0.f;
    float *C = reinterpret_cast<float *>(g.C) + (int64_t)m * g.scm + (int64_t)n * g.scn;
    if (g.accumulate)
        *C += v;
    else
        *C = v;
}

// Operand mode (see stage_load) from the strides and the base alignment.
// The vector modes read whole 8-element segments, so they also need every
// segment that starts inside the operand to end inside its row: K <= sr for
// mode 0, R <= sk for mode 1 (both strides multiples of 8).
static int operand_mode(const bf16 *p, int64_t sr, int64_t sk, int R, int K) {
    const bool aligned = (((uintptr_t)p) & 15) == 0;
    if (aligned && sk == 1 && sr % 8 == 0 && K <= sr) return 0;
    if (aligned && sr == 1 && sk % 8 == 0 && R <= sk) return 1;
    return 2;
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
    const bool parts = g.ksplit > 1 || g.keep_parts;
    if (parts && (g.bias || g.relu || g.gate || g.out_bf16 || !g.part || g.colpart || g.lossx ||
                  (int64_t)g.M * g.N > INT32_MAX))
        return hipErrorInvalidValue;
    if (g.lossx && (!g.lossfree || !g.losspart || g.relu || g.gate || g.accumulate)) return hipErrorInvalidValue;
    if (g.colpart && g.accumulate) return hipErrorInvalidValue;
    const int z = g.ksplit > 1 ? g.ksplit : 1;
    // 64 x 64 tiles: the products of the networks the proposal accepts
    // (H <= 2,496, training batches <= 16,384, scored batches <= 65,536)
    // have at most sixteen 128 x 128 tiles per CU, where four 64 x 64
    // workgroups per CU ran faster (a 16,384 x 1,024 product: 49 us against
    // 52 us)
    constexpr int TT = 64;
    const int tiles = ((g.N + TT - 1) / TT) * ((g.M + TT - 1) / TT);
    dim3 grid(8 * ((tiles + 7) / 8), 1, z);
    const int ma = operand_mode(g.A, g.sam, g.sak, g.M, g.K), mb = operand_mode(g.B, g.sbn, g.sbk, g.N, g.K);
    if (g.kperm && (ma != 0 || mb != 0)) return hipErrorInvalidValue;
    const void *fn = nullptr;
#define PBIT_GEMM(A_, B_) \
    if (ma == A_ && mb == B_)  \
        fn = (const void *)gemm_kernel<A_, B_, TT>;
    PBIT_GEMM(0, 0) PBIT_GEMM(0, 1) PBIT_GEMM(0, 2)
    PBIT_GEMM(1, 0) PBIT_GEMM(1, 1) PBIT_GEMM(1, 2)
    PBIT_GEMM(2, 0) PBIT_GEMM(2, 1) PBIT_GEMM(2, 2)
#undef PBIT_GEMM
    void *args[] = {const_cast<GemmArgs *>(&g)};
    hipError_t e = hipLaunchKernel(fn, grid, dim3(256), args, 0, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess || g.ksplit <= 1 || g.keep_parts) return e;
    const int64_t tot = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// element-wise helpers
// ---------------------------------------------------------------------------
// Lattice words (word-major, word w of sample b at states[w n + b]) -> bf16
// 0/1 rows X[b][i], zero for i >= D.
hipError_t launch_gemm_group(const GemmArgs *gs, int count, hipStream_t s) {
    if (count < 1 || count > GEMM_GROUP_MAX) return hipErrorInvalidValue;
    GemmGroup gg;
    std::memset(&gg, 0, sizeof(gg));
    gg.count = count;
    int ma = -1, mb = -1;
    int64_t blocks = 0;
    for (int i = 0; i < count; ++i) {
        const GemmArgs &g = gs[i];
        // slices kept for a later finalize: no epilogue, no reduction launch
        if (!g.keep_parts || !g.part || g.bias || g.relu || g.gate || g.out_bf16 || g.colpart || g.lossx || g.kperm ||
            (int64_t)g.M * g.N > INT32_MAX)
            return hipErrorInvalidValue;
        const int a = operand_mode(g.A, g.sam, g.sak, g.M, g.K), b = operand_mode(g.B, g.sbn, g.sbk, g.N, g.K);
        if (i == 0) {
            ma = a;
            mb = b;
        } else if (a != ma || b != mb) {
            // operand layouts differ: a launch each, same slices
            for (int j = 0; j < count; ++j) {
                const hipError_t e = launch_gemm(gs[j], s);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        }
        const int tiles = ((g.N + 63) / 64) * ((g.M + 63) / 64);
        gg.g[i] = g;
        gg.bx[i] = 8 * ((tiles + 7) / 8);
        gg.z[i] = g.ksplit > 1 ? g.ksplit : 1;
        blocks += (int64_t)gg.bx[i] * gg.z[i];
    }
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    const void *fn = nullptr;
#define PBIT_GEMM(A_, B_) \
    if (ma == A_ && mb == B_) \
        fn = (const void *)gemm_group_kernel<A_, B_>;
    PBIT_GEMM(0, 0) PBIT_GEMM(0, 1) PBIT_GEMM(0, 2)
    PBIT_GEMM(1, 0) PBIT_GEMM(1, 1) PBIT_GEMM(1, 2)
    PBIT_GEMM(2, 0) PBIT_GEMM(2, 1) PBIT_GEMM(2, 2)
#undef PBIT_GEMM
    void *args[] = {&gg};
    hipError_t e = hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(256), args, 0, s);
    if (e == hipSuccess) e = hipGetLastError();
    return e;
}

__global__ void unpack_kernel(const uint32_t *__restrict__ states, int n, int D, int DP, bf16 *__restrict__ X) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * DP) return;
    const int b = (int)(e / DP), i = (int)(e % DP);
    float v = 0.f;
    if (i < D) v = (float)((states[(int64_t)(i >> 5) * n + b] >> (i & 31)) & 1u);
    X[e] = (bf16)v;
}

// Block 0 of a finalize launch adds the loss shares in a fixed order.
__device__ __forceinline__ void gf_loss(const GradFinal &a) {
    __shared__ float red[256];
    float v = 0.f;
    for (int i = threadIdx.x; i < a.nloss; i += 256) v += a.losspart[i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *a.loss = red[0];
}

// The gradient of flat parameter i < P: a weight's split-K slices added in
// ascending order and masked by degree, a bias's 64-row column partials
// added in ascending order.
__device__ __forceinline__ float gf_grad(const GradFinal &a, int64_t i) {
    const int D = a.D, H = a.H;
    auto slices = [&](const float *part, int z, int64_t MN, int64_t e) {
        float v = 0.f;
#pragma unroll 4
        for (int k = 0; k < z; ++k) v += part[(int64_t)k * MN + e];
        return v;
    };
    // (unrolled so a thread's chunk loads are in flight together: the bias
    // entries' threads would otherwise wait one memory latency per chunk)
    auto cols = [&](const float *part, int N, int j) {
        float v = 0.f;
#pragma unroll 16
        for (int k = 0; k < a.chunks; ++k) v += part[(int64_t)k * N + j];
        return v;
    };
    if (i < a.ob1) {  // W1 [D][H]
        const int64_t e = i - a.oW1;
        const int m = (int)(e / H), n = (int)(e - (int64_t)m * H);
        return a.deg_in[m] > a.deg1[n] ? 0.f : slices(a.pW1, a.zW1, (int64_t)D * H, e);
    } else if (i < a.oW2) {  // b1
        return cols(a.cb1, H, (int)(i - a.ob1));
    } else if (i < a.ob2) {  // W2 [H][H]
        const int64_t e = i - a.oW2;
        const int m = (int)(e / H), n = (int)(e - (int64_t)m * H);
        return a.deg1[m] > a.deg2[n] ? 0.f : slices(a.pW2, a.zW2, (int64_t)H * H, e);
    } else if (i < a.oV) {  // b2
        return cols(a.cb2, H, (int)(i - a.ob2));
    } else if (i < a.oc) {  // V [H][D]
        const int64_t e = i - a.oV;
        const int m = (int)(e / D), n = (int)(e - (int64_t)m * D);
        return a.deg2[m] > a.deg_out[n] ? 0.f : slices(a.pV, a.zV, (int64_t)H * D, e);
    }
    return cols(a.cc, D, (int)(i - a.oc));  // c
}

// One Adam step from gradient gi, moments m, v and value th (updated in
// place).
__device__ __forceinline__ void gf_adam_math(const GradFinal &a, float gi, float &m, float &v, float &th) {
    m = a.b1 * m + (1.f - a.b1) * gi;
    v = a.b2 * v + (1.f - a.b2) * gi * gi;
    th = th - a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
}

// One Adam step of parameter i on gradient gi; returns the new value.
__device__ __forceinline__ float gf_adam(const GradFinal &a, int64_t i, float gi) {
    float m = a.m[i], v = a.v[i], th = a.th[i];
    gf_adam_math(a, gi, m, v, th);
    a.m[i] = m;
    a.v[i] = v;
    a.th[i] = th;
    return th;
}

// The gradient of every parameter from what the training GEMMs left, then
// either stored (adam == 0) or taken by one Adam step; block 0 also adds the
// loss shares.  One thread per flat parameter.
__global__ __launch_bounds__(256) void grad_final_kernel(GradFinal a) {
    if (blockIdx.x == 0 && a.loss) gf_loss(a);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.P) return;
    const float gi = gf_grad(a, i);
    if (!a.adam)
        a.grad[i] = gi;
    else
        (void)gf_adam(a, i, gi);
}

// The Adam step with the bf16 shadows of the updated weights written in the
// same pass (the arithmetic of grad_final_kernel, element for element).  The
// first tiles.x + tiles.y + tiles.z workgroups take 32 x 32 tiles of W1, W2
// and V (rows k0.. of the KP rows of WT, columns n0..): thread (column tx,
// row group ty) updates rows ty, ty + 8, ... and writes Wb along n; the tile
// is transposed through LDS and WT written along k, zero past K.  The next
// ceil((2H + D) / 256) take the biases b1, b2, c, one thread each, and the
// rest, when a.ux_n > 0, unpack the next batch (unpack_row8).  Workgroup 0
// adds the loss shares.
constexpr int AS_ROWS = 32, AS_COLS = 32;
__global__ __launch_bounds__(256) void adam_shadow_kernel(GradFinal a, int4 tiles) {
    if (blockIdx.x == 0 && a.loss) gf_loss(a);
    int id = (int)blockIdx.x;
    const int tcount[3] = {tiles.x, tiles.y, tiles.z};
    const int64_t off[3] = {a.oW1, a.oW2, a.oV};
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        if (id < tcount[w]) {
            __shared__ float t[AS_ROWS][AS_COLS + 1];
            const ShadowJob &J = a.sh[w];
            const int gx = (J.N + AS_COLS - 1) / AS_COLS;
            const int n0 = (id % gx) * AS_COLS, k0 = (id / gx) * AS_ROWS;
            const int tx = threadIdx.x & (AS_COLS - 1), ty = threadIdx.x / AS_COLS;
            constexpr int RG = 256 / AS_COLS, Q = AS_ROWS / RG;
            // every load of the thread's elements first, then the arithmetic
            // and the stores (the stores could alias the loads, so
            // interleaved they would wait one memory latency apiece)
            float g[Q], m[Q], v[Q], th[Q];
            const int n = n0 + tx;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int k = k0 + ty + RG * q;
                g[q] = m[q] = v[q] = th[q] = 0.f;
                if (k < J.K && n < J.N) {
                    const int64_t i = off[w] + (int64_t)k * J.N + n;
                    g[q] = gf_grad(a, i);
                    m[q] = a.m[i];
                    v[q] = a.v[i];
                    th[q] = a.th[i];
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int k = k0 + ty + RG * q;
                float x = 0.f;
                if (k < J.K && n < J.N) {
                    const int64_t e = (int64_t)k * J.N + n, i = off[w] + e;
                    gf_adam_math(a, g[q], m[q], v[q], th[q]);
                    a.m[i] = m[q];
                    a.v[i] = v[q];
                    a.th[i] = th[q];
                    J.Wb[e] = (bf16)th[q];
                    x = th[q];
                }
                t[ty + RG * q][tx] = x;
            }
            __syncthreads();
            // transposed: thread (k offset kx, column group ny) writes
            // WT[n0 + ny + 8 r][k0 + kx]
            const int kx = threadIdx.x & (AS_ROWS - 1), ny = threadIdx.x / AS_ROWS;
#pragma unroll
            for (int r = 0; r < AS_COLS / 8; ++r) {
                const int nn = n0 + ny + 8 * r, k = k0 + kx;
                if (nn < J.N && k < J.KP) J.WT[(int64_t)nn * J.KP + k] = (bf16)t[kx][ny + 8 * r];
            }
            return;
        }
        id -= tcount[w];
    }
    // biases: b1 [H], b2 [H], c [D] in that order
    const int nbias = (2 * a.H + a.D + 255) / 256;
    if (id < nbias) {
        const int j = id * 256 + (int)threadIdx.x;
        int64_t i;
        if (j < a.H)
            i = a.ob1 + j;
        else if (j < 2 * a.H)
            i = a.ob2 + (j - a.H);
        else if (j < 2 * a.H + a.D)
            i = a.oc + (j - 2 * a.H);
        else
            return;
        (void)gf_adam(a, i, gf_grad(a, i));
        return;
    }
    // the next batch's unpack
    const uint32_t e = (uint32_t)(id - nbias) * 256u + threadIdx.x;
    if (e < (uint32_t)a.ux_n * ((uint32_t)a.ux_DP >> 3)) unpack_row8(a.ux_states, a.ux_stride, a.ux_b0, a.D, a.ux_DP, a.ux_X, e);
}

// The ReLU-derivative gate of a library product's bf16 output and its column
// partials: G[m][j] = 0 where A[m][j] <= 0, then per 64-row chunk c the column
// sums of the gated G into colpart[c N + j].  A workgroup takes 64 rows x 128
// columns; thread (column group of 8, row group of 4) adds its 4 rows in
// ascending order, and the 16 row groups are added in order.  N % 8 == 0 and
// 16-byte aligned rows.
__global__ __launch_bounds__(256) void gate_colsum_kernel(bf16 *__restrict__ G, const bf16 *__restrict__ A, int n,
                                                          int N, float *__restrict__ colpart) {
    __shared__ float red[16][128];
    const int cg = threadIdx.x & 15, rg = threadIdx.x >> 4;
    const int c0 = blockIdx.x * 128 + cg * 8;
    const int r0 = blockIdx.y * 64 + rg * 4;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (c0 < N) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + q;
            if (r < n) {
                const int64_t o = (int64_t)r * N + c0;
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(A + o);
                bf16x8 g = *reinterpret_cast<const bf16x8 *>(G + o);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    if (!((float)a[i] > 0.f)) g[i] = (bf16)0.f;
                    acc[i] += (float)g[i];
                }
                *reinterpret_cast<bf16x8 *>(G + o) = g;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) red[rg][cg * 8 + i] = acc[i];
    __syncthreads();
    const int j = blockIdx.x * 128 + (int)threadIdx.x;
    if (threadIdx.x < 128 && j < N) {
        float v = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) v += red[q][threadIdx.x];
        colpart[(int64_t)blockIdx.y * N + j] = v;
    }
}

// bf16 shadows of up to three K x N weights (row-major) and their transposes
// N x KP (row n holds the K inputs of unit n, zero-padded to KP), one weight
// per blockIdx.z.  Workgroup (blockIdx.x, blockIdx.y) takes the 32 x 32 tile
// of columns n0.. and rows k0..: rows are read and Wb written along n, the
// tile is transposed through LDS and WT written along k.
__global__ __launch_bounds__(256) void shadow_kernel(ShadowJobs jobs) {
    __shared__ float t[32][33];
    const ShadowJob &J = jobs.j[blockIdx.z];
    const int n0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
    if (n0 >= J.N || k0 >= J.KP) return;  // whole workgroup: a smaller weight
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int r = ty; r < 32; r += 8) {
        const int k = k0 + r, n = n0 + tx;
        float w = 0.f;
        if (k < J.K && n < J.N) {
            w = J.W[(int64_t)k * J.N + n];
            J.Wb[(int64_t)k * J.N + n] = (bf16)w;
        }
        t[r][tx] = w;
    }
    __syncthreads();
#pragma unroll
    for (int r = ty; r < 32; r += 8) {
        const int n = n0 + r, k = k0 + tx;
        if (n < J.N && k < J.KP) J.WT[(int64_t)n * J.KP + k] = (bf16)t[tx][r];
    }
}

// ---------------------------------------------------------------------------
// log q of given paths (score mode)
// ---------------------------------------------------------------------------
// Workgroup of 256 threads per 64 paths.  Free positions are taken in
// chunks of 64: all threads compute the chunk's terms log q_f (thread t: the
// position t % 64 of paths t / 64, t / 64 + 4, ...; a wave reads 64
// positions of one logit row), then thread c < 64 adds path c's terms in
// ascending position order, the order of the sampler's accumulation.
__global__ __launch_bounds__(256) void logq_kernel(const float *__restrict__ L, const uint32_t *__restrict__ states,
                                                   uint64_t stride, uint64_t b0, const int *__restrict__ fpos, int h,
                                                   int n, int D, double *__restrict__ out) {
    __shared__ double term[64][65];
    const int cb = blockIdx.x * 64, t = threadIdx.x;
    double s = 0.0;
    for (int f0 = 0; f0 < h; f0 += 64) {
        const int nf = min(64, h - f0), f = t & 63;
        if (f < nf) {
            const int p = fpos[f0 + f];
            for (int c = t >> 6; c < 64; c += 4) {
                const int b = cb + c;
                if (b < n) {
                    const uint32_t x = (states[(uint64_t)(p >> 5) * stride + b0 + b] >> (p & 31)) & 1u;
                    term[c][f] = made_log_prob(made_threshold(L[(int64_t)b * D + p]), x);
                }
            }
        }
        __syncthreads();
        if (t < 64 && cb + t < n)
            for (int j = 0; j < nf; ++j) s += term[t][j];
        __syncthreads();
    }
    if (t < 64 && cb + t < n) out[cb + t] = s;
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
    const int DP = a.DP, H = a.H, W = a.W, h = a.h;
    // LDS rows padded by 8 elements (16 bytes): rows of 1,024 bf16 are a
    // multiple of the 64 four-byte banks, and the 16 rows a half tile reads
    // at once would otherwise sit on one bank
    const int XS = DP + 8, HS = H + 8;
    bf16 *Xs = reinterpret_cast<bf16 *>(smem);           // [CS][XS]
    bf16 *H1s = Xs + CS * XS;                             // [CS][HS]
    bf16 *H2s = H1s + CS * HS;                             // [CS][HS]
    float *logit = reinterpret_cast<float *>(H2s + CS * HS);  // [CS]
    uint32_t *lat = reinterpret_cast<uint32_t *>(logit + CS);  // [CS][W]
    uint32_t *Ts = lat + CS * W;                          // deferred: [h][CS] thresholds
    uint32_t *cones = Ts + (a.defer ? h * CS : 0);        // deferred: [h][W] cone words
    // deferred: [h][CS] log-probabilities, over the dead activations when they fit
    double *lgs = reinterpret_cast<double *>(a.defer == 2 ? (void *)H1s
                                                          : (void *)(cones + (a.defer ? ((h * W + 1) & ~1) : 0)));
    const int lane = threadIdx.x;
    const int c0 = blockIdx.x * CS;
    const uint32_t *B = a.blob;
    const uint32_t *cw = B + B[H_OFF_CONST];
    const uint32_t *cone_g = B + B[H_OFF_CONE];
    const uint32_t WS = B[H_WS];
    const uint32_t cid = B[H_CID];

    for (int e = lane; e < CS * XS; e += 64) {
        const int i = e % XS;
        Xs[e] = (bf16)((i < a.D) ? (float)((cw[i >> 5] >> (i & 31)) & 1u) : 0.f);
    }
    for (int e = lane; e < 2 * CS * HS; e += 64) H1s[e] = (bf16)0.f;
    for (int e = lane; e < CS * W; e += 64) lat[e] = cw[e % W];
    if (a.defer)
        for (int e = lane; e < h * W; e += 64) cones[e] = cone_g[(int64_t)(e / W) * WS + e % W];
    __syncthreads();
    double lq = 0.0;
    U4 u4 = {0u, 0u, 0u, 0u};
    const int row = lane & 15, kq = (lane >> 4) * 8;
    for (int f = 0; f < h; ++f) {
        const int4 ph = a.phase[f];  // {u1a, u1b, u2a, u2b}
        const int4 kk = a.phase_k[f];  // {K1 end, K2 end, K3 end, position p}
        const int p = kk.w;
        // (a) first-layer units whose degree became <= p
        for (int u0 = ph.x; u0 < ph.y; u0 += 16) {
            const int u = min(u0 + row, H - 1);
            const f32x4 acc = mfma_chunks(Xs + row * XS + kq, a.W1T + (int64_t)u * DP + kq, (kk.x + 31) / 32);
            const int un = u0 + row;
            if (un < ph.y) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = acc[e] + a.b1[un];
                    v = v > 0.f ? v : 0.f;
                    H1s[((lane >> 4) * 4 + e) * HS + un] = (bf16)v;
                }
            }
        }
        __syncthreads();
        // (b) second-layer units whose degree became <= p
        for (int u0 = ph.z; u0 < ph.w; u0 += 16) {
            const int u = min(u0 + row, H - 1);
            const f32x4 acc = mfma_chunks(H1s + row * HS + kq, a.W2T + (int64_t)u * H + kq, (kk.y + 31) / 32);
            const int un = u0 + row;
            if (un < ph.w) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = acc[e] + a.b2[un];
                    v = v > 0.f ? v : 0.f;
                    H2s[((lane >> 4) * 4 + e) * HS + un] = (bf16)v;
                }
            }
        }
        __syncthreads();
        // (c) logit of position p (every column of the tile computes it)
        {
            const f32x4 acc = mfma_chunks(H2s + row * HS + kq, a.VT + (int64_t)p * H + kq, (kk.z + 31) / 32);
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
                    // one Philox block serves four consecutive free bits
                    if ((f & 3) == 0)
                        u4 = philox4x32_10(a.step, (uint32_t)f >> 2, a.chain_begin + chain, cid | (1u << 16),
                                           a.seed_lo, a.seed_hi);
                    const uint32_t u = (f & 3) == 0 ? u4.x : ((f & 3) == 1 ? u4.y : ((f & 3) == 2 ? u4.z : u4.w));
                    bit = u < T ? 1u : 0u;
                }
                if (a.defer)
                    Ts[f * CS + lane] = T;
                else
                    lq += made_log_prob(T, bit);
                // the lattice bit at p is the free bit itself: flip its cone
                // when the drawn value differs from the current one
                const uint32_t cur = (lat[lane * W + (p >> 5)] >> (p & 31)) & 1u;
                if (bit != cur) {
                    for (int w = 0; w < W; ++w) {
                        // the cone from LDS or from the image, each by its own
                        // load (not a generic one)
                        typedef const __attribute__((address_space(3))) uint32_t lds_u32;
                        uint32_t mw = a.defer ? ((lds_u32 *)cones)[f * W + w] : cone_g[(int64_t)f * WS + w];
                        lat[lane * W + w] ^= mw;
                        while (mw) {
                            const int i = 32 * w + __builtin_ctz(mw);
                            mw &= mw - 1;
                            const float xv = (float)Xs[lane * XS + i];
                            Xs[lane * XS + i] = (bf16)(1.f - xv);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (a.defer) {
        // every lane computes log-probabilities (four lanes per chain), then
        // each chain sums its own in free-bit order, as the batched scorer does
        const int c = lane & 15;
        const int chain = c0 + c;
        if (chain < a.n) {
            for (int f = lane >> 4; f < h; f += 4) {
                const int p = a.phase_k[f].w;
                const uint32_t bit = (lat[c * W + (p >> 5)] >> (p & 31)) & 1u;
                lgs[f * CS + c] = made_log_prob(Ts[f * CS + c], bit);
            }
        }
        __syncthreads();
        if (lane < CS && chain < a.n)
            for (int f = 0; f < h; ++f) lq += lgs[f * CS + lane];
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

// ---------------------------------------------------------------------------
// register-resident sampler for small networks
// ---------------------------------------------------------------------------
// The same autoregressive procedure for H <= 256 and lattices of at most 256
// bits, with every activation kept in registers and the network in LDS.
// Each product is taken transposed: the weight rows of 16 units are the
// MFMA's A operand and 16 chains (one slot, below) its B operand, so the outputs of
// a unit land in the lanes of their chain (lane & 15) and feed the next
// product as its B operand directly.  Half t of K-chunk cc is the tile of
// the 16 consecutive units 32 cc + 16 t + r (row r): lane group g receives
// units 32 cc + 16 t + 4 g + e (e = 0..3), and supplies them as elements
// 4 t + e of its 8-element B slice of the chunk, so no lane exchange is
// needed; the next product's weights are staged with the matching order of
// K inside each 32-unit chunk (k-slot 8 g + 4 t + e holds unit 16 t + 4 g +
// e).  Units are sorted by degree, so a phase's few new units usually sit in
// one half tile.  A tile is computed when it holds a unit whose degree falls
// in the current phase (the host lists them per free bit; see layer_tiles
// for why writing all 16 of its units is safe).
//
// A wave carries NP paths per chain through the same tiles: NP = 1 samples
// (or, with `score`, scores) one path; NP = 2 samples the proposal (path 0)
// and scores the chain's current path (path 1, from `score`) in one pass, the
// weight rows and tile decisions shared.  Every path's arithmetic is the one
// the single-path kernel performs, so the results are the same bits.

__device__ __forceinline__ bf16x8 bits_to_bf16x8(uint32_t b) {
    // element s is 1.0 (0x3f80) when bit s of b is set, else 0
    u32x4v d;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        d[j] = ((b >> (2 * j)) & 1u) * 0x3f80u | ((b >> (2 * j + 1)) & 1u) * 0x3f800000u;
    return __builtin_bit_cast(bf16x8, d);
}

template <int N>
__device__ __forceinline__ uint32_t pick_word(const uint32_t (&v)[N], int i) {
    uint32_t r = 0u;
#pragma unroll
    for (int w = 0; w < N; ++w) r = (w == i) ? v[w] : r;
    return r;
}

// this lane's 8-element slices of chunks k < nk of one weight row (LDS)
template <int N>
__device__ __forceinline__ void load_rows(bf16x8 (&av)[N], const bf16 *__restrict__ wrow, int nk) {
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k < nk) av[k] = *reinterpret_cast<const bf16x8 *>(wrow + 32 * k);
}

// sum over chunks k < nk (ascending, from zero) of A = av[k] times B = ops[k]
// (8 bf16 per lane, as bf16x8 or as four dwords)
template <int N, class Op>
__device__ __forceinline__ f32x4 mfma_ops(const bf16x8 (&av)[N], const Op (&ops)[N], int nk) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (k < nk)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[k], __builtin_bit_cast(bf16x8, ops[k]), acc, 0, 0, 0);
    return acc;
}

typedef bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float relu(float v) { return v > 0.f ? v : 0.f; }

// two floats as a dword of two bf16 (element 0 in the low half)
__device__ __forceinline__ uint32_t pack_bf16(float x, float y) {
    const f32x2 v = {x, y};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// one layer's phase for NP paths: the half tiles flagged in `tiles` (bit
// 2 cc + t; the host sets those that hold a unit whose degree falls in this
// phase) from ops (nk chunks) and the rows of WT (row stride rs), bias, ReLU,
// written into act (chunk cc: four dwords, element s of the lane's 8-element
// slice in the half s & 1 of dword s >> 1).  All 16 units of a tile are
// written.  The new ones are what they must be; the earlier ones come out
// with the bits they already had (their inputs are final and the extra K
// chunks add exact zeros); the later ones are provisional until their own
// phase recomputes them, and until then they only meet weights the degree
// masks keep at exactly zero (a ReLU output is finite and >= 0, so each such
// product is +0).  The chunk loop is unrolled so every write goes to a fixed
// register.
template <int NP, int NO, int NA, class OpFn>
__device__ __forceinline__ void layer_tiles(u32x4v (&act)[NP][NA], OpFn op, const bf16 *__restrict__ WT, int rs,
                                            const float *__restrict__ bias, uint32_t tiles, int nk, int g, int rrow) {
#pragma unroll
    for (int cc = 0; cc < NA; ++cc) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (!(tiles & (1u << (2 * cc + t)))) continue;
            bf16x8 av[NO];
            load_rows<NO>(av, WT + (int64_t)(32 * cc + 16 * t + rrow) * rs + 8 * g, nk);
            const float4 bb = *reinterpret_cast<const float4 *>(bias + 32 * cc + 16 * t + 4 * g);
            // per path, the sum over chunks k < nk (ascending, from zero) of
            // av[k] times its B slice op(q, k); one branch per chunk for all
            // paths, and a listed tile always has nk >= 1
            f32x4 acc[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q)
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], op(q, 0), f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
            for (int k = 1; k < NO; ++k) {
                if (k < nk) {
#pragma unroll
                    for (int q = 0; q < NP; ++q)
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[k], op(q, k), acc[q], 0, 0, 0);
                }
            }
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                act[q][cc][2 * t] = pack_bf16(relu(acc[q][0] + bb.x), relu(acc[q][1] + bb.y));
                act[q][cc][2 * t + 1] = pack_bf16(relu(acc[q][2] + bb.z), relu(acc[q][3] + bb.w));
            }
        }
    }
}

// LDS image of the network for the register-resident sampler: the table of
// 8-bit input slices as bf16x8 (256 x 16 bytes), W1T (H rows of DP), W2T (H
// rows of H), VT (D rows of H) as bf16, each row padded by 8 elements so the
// 16 rows a half tile reads at once fall on different LDS banks, then b1, b2
// (H each) and c (D) as FP32.
constexpr int REG_PAD = 8;

struct RegLayout {
    size_t lut, w1, w2, v, b1, b2, c, total;
};

__host__ __device__ inline RegLayout reg_layout(int D, int DP, int H) {
    RegLayout L;
    L.lut = 0;
    L.w1 = 256 * 16;
    L.w2 = L.w1 + (size_t)H * (DP + REG_PAD) * 2;
    L.v = L.w2 + (size_t)H * (H + REG_PAD) * 2;
    L.b1 = (L.v + (size_t)D * (H + REG_PAD) * 2 + 15) & ~(size_t)15;
    L.b2 = L.b1 + (size_t)H * 4;
    L.c = L.b2 + (size_t)H * 4;
    L.total = (L.c + (size_t)D * 4 + 15) & ~(size_t)15;
    return L;
}

// copies n bytes (a multiple of 16, both ends 16-byte aligned) into LDS
__device__ __forceinline__ void stage16(unsigned char *dst, const void *src, size_t n) {
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
    uint4 *d4 = reinterpret_cast<uint4 *>(dst);
    for (size_t i = threadIdx.x; i < n / 16; i += blockDim.x) d4[i] = s4[i];
}

// copies `rows` bf16 rows of `len` elements (a multiple of 8) into LDS rows
// of len + REG_PAD elements; eight loads per thread are in flight at once, so
// a small workgroup is not held up by one memory latency per piece
__device__ __forceinline__ void stage_rows(unsigned char *dst, const bf16 *src, int rows, int len) {
    const int q = len / 8;  // 16-byte pieces per row
    const int n = rows * q;
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
    constexpr int U = 8;
    for (int i0 = threadIdx.x; i0 < n; i0 += U * blockDim.x) {
        uint4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < n) v[u] = s4[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < n) *reinterpret_cast<uint4 *>(dst + ((size_t)(i / q) * (len + REG_PAD) + 8 * (i % q)) * 2) = v[u];
        }
    }
}

// A wave carries S = NB x NP slots of 16 chains: NB blocks of chains, each
// with NP paths (path 0 drawn, or scored when only `score` is given; with
// NP = 2 path 1 is the scored current path).  Slot s = q NB + j holds path q
// of chains 16 j + c (c = lane & 15) of the wave.  Every lane keeps the
// activations and lattices of all S slots for its c, so each slot's products
// take the same weight rows; the per-chain work of a position (threshold,
// draw or read of the bit, logarithm) is done by lane group g for slot
// g % S, and one ballot hands every slot's bits to all lanes.  With S = 4
// each lane does one chain-path, so nothing is repeated.
// FULL (rows exactly NX and NH chunks long: DP = 32 NX, H = 32 NH): every
// product runs over all chunks of its rows instead of the phase's K range.
// The extra chunks multiply weights the degree masks keep at exactly zero,
// so the units a phase keeps come out with the same bits, and the products
// need no per-chunk branches.
// stage_rows for rows whose K runs over hidden units: inside each 32-unit
// chunk, k-slot 8 g + 4 t + e takes unit 16 t + 4 g + e (the order in which
// the half tiles hand their outputs to the lane groups), moved as 8-byte
// pieces of four units
__device__ __forceinline__ void stage_rows_k(unsigned char *dst, const bf16 *src, int rows, int len) {
    const int q = len / 4;  // 8-byte pieces per row
    const int n = rows * q;
    const uint2 *s2 = reinterpret_cast<const uint2 *>(src);
    constexpr int U = 8;
    for (int i0 = threadIdx.x; i0 < n; i0 += U * blockDim.x) {
        uint2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < n) v[u] = s2[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * blockDim.x;
            if (i < n) {
                const int r = i / q, pc = i % q;       // source piece: units 4 pc .. 4 pc + 3
                const int cc = pc >> 3, w = pc & 7;    // chunk, piece in chunk: units 4 w .. (w = 4 t + g)
                const int t = w >> 2, g = w & 3;
                const int slot = 32 * cc + 8 * g + 4 * t;  // its k-slots
                *reinterpret_cast<uint2 *>(dst + ((size_t)r * (len + REG_PAD) + slot) * 2) = v[u];
            }
        }
    }
}

template <int NX, int NH, int NB, int NP, bool FULL>
__global__ __launch_bounds__(512) void made_sample_reg_kernel(SampleArgs a) {
    constexpr int S = NB * NP;
    extern __shared__ __align__(16) unsigned char smem[];
    const int h = a.h, W = a.W, DP = a.DP, H = a.H, D = a.D;
    const RegLayout L = reg_layout(D, DP, H);
    // the whole network goes to LDS once per workgroup; after this barrier
    // every wave runs on its own
    stage_rows(smem + L.w1, a.W1T, H, DP);
    stage_rows_k(smem + L.w2, a.W2T, H, H);
    stage_rows_k(smem + L.v, a.VT, D, H);
    stage16(smem + L.b1, a.b1, (size_t)H * 4);
    stage16(smem + L.b2, a.b2, (size_t)H * 4);
    {
        float *cl = reinterpret_cast<float *>(smem + L.c);
        for (int i = threadIdx.x; i < D; i += blockDim.x) cl[i] = a.c[i];
        bf16x8 *lut = reinterpret_cast<bf16x8 *>(smem + L.lut);
        for (int i = threadIdx.x; i < 256; i += blockDim.x) lut[i] = bits_to_bf16x8((uint32_t)i);
    }
    __syncthreads();
    const bf16x8 *lut = reinterpret_cast<const bf16x8 *>(smem + L.lut);
    const bf16 *W1s = reinterpret_cast<const bf16 *>(smem + L.w1);
    const bf16 *W2s = reinterpret_cast<const bf16 *>(smem + L.w2);
    const bf16 *Vs = reinterpret_cast<const bf16 *>(smem + L.v);
    const float *b1s = reinterpret_cast<const float *>(smem + L.b1);
    const float *b2s = reinterpret_cast<const float *>(smem + L.b2);
    const float *cs = reinterpret_cast<const float *>(smem + L.c);

    const int lane = threadIdx.x & 63;
    const int c = lane & 15, g = lane >> 4;
    const int base = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16 * NB;  // first chain of the wave
    if (__builtin_amdgcn_readfirstlane(base) >= a.n) return;  // the wave has no chain
    // this lane's slot for the per-chain work
    const int my_s = g % S, my_q = my_s / NB;
    const int my_chain = base + 16 * (my_s % NB) + c;
    const bool my_valid = my_chain < a.n;
    // path q draws its bits unless it is the scored one (the last path when
    // `score` is given)
    const int qs = a.score ? NP - 1 : NP;  // first scored path (NP: none)
    const bool my_draws = my_q < qs;
    const uint32_t *B = a.blob;
    const uint32_t *cw = B + B[H_OFF_CONST];
    const uint32_t cid = B[H_CID];

    uint32_t lat[S][NX], path[NX];
    u32x4v act1[S][NH], act2[S][NH];
#pragma unroll
    for (int w = 0; w < NX; ++w)
        path[w] = (!my_draws && my_valid && w < W) ? a.score[(int64_t)w * a.n + my_chain] : 0u;
#pragma unroll
    for (int q = 0; q < S; ++q) {
#pragma unroll
        for (int w = 0; w < NX; ++w) lat[q][w] = w < W ? cw[w] : 0u;
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            act1[q][k] = u32x4v{0u, 0u, 0u, 0u};
            act2[q][k] = u32x4v{0u, 0u, 0u, 0u};
        }
    }
    double lq = 0.0;
    const int rrow = c;  // this lane's A row within a half tile
    U4 u4 = {0u, 0u, 0u, 0u};
    for (int f = 0; f < h; ++f) {
        const uint32_t *rec = a.sched + (size_t)f * 16;  // wave-uniform: one scalar load
        const uint32_t t1 = rec[4] & 0xffffu, t2 = rec[5] & 0xffffu;
        const int nk1 = FULL ? NX : (int)(rec[4] >> 16), nk2 = FULL ? NH : (int)(rec[5] >> 16);
        const int nk3 = FULL ? NH : (int)rec[6], p = (int)rec[7];
        // layer 1 reads its input slices (8 lattice bits as bf16) from the
        // table as it goes; layer 2 reads the layer-1 activations
        if (t1)
            layer_tiles<S, NX, NH>(
                act1, [&](int q, int k) { return lut[(lat[q][k] >> (8 * g)) & 0xffu]; }, W1s, DP + REG_PAD, b1s, t1,
                nk1, g, rrow);
        if (t2)
            layer_tiles<S, NH, NH>(
                act2, [&](int q, int k) { return __builtin_bit_cast(bf16x8, act1[q][k]); }, W2s, H + REG_PAD, b2s,
                t2, nk2, g, rrow);
        // logits of position p: every A row is row p of V, so all four
        // accumulator elements of a slot hold its chains' logits
        bf16x8 vv[NH];
        load_rows<NH>(vv, Vs + (int64_t)p * (H + REG_PAD) + 8 * g, nk3);
        float lg = 0.f;
        if (nk3 > 0) {
            f32x4 lacc[S];
#pragma unroll
            for (int q = 0; q < S; ++q)
                lacc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vv[0], __builtin_bit_cast(bf16x8, act2[q][0]),
                                                                  f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
            for (int k = 1; k < NH; ++k) {
                if (k < nk3) {
#pragma unroll
                    for (int q = 0; q < S; ++q)
                        lacc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vv[k], __builtin_bit_cast(bf16x8, act2[q][k]),
                                                                          lacc[q], 0, 0, 0);
                }
            }
#pragma unroll
            for (int q = 0; q < S; ++q) lg = (q == my_s) ? lacc[q][0] : lg;
        }
        const uint32_t T = made_threshold(lg + cs[p]);
        uint32_t bit;
        if (my_draws) {
            if ((f & 3) == 0)
                u4 = philox4x32_10(a.step, (uint32_t)f >> 2, a.chain_begin + (uint32_t)my_chain, cid | (1u << 16),
                                   a.seed_lo, a.seed_hi);
            const uint32_t u = (f & 3) == 0 ? u4.x : ((f & 3) == 1 ? u4.y : ((f & 3) == 2 ? u4.z : u4.w));
            bit = u < T ? 1u : 0u;
        } else {
            bit = (pick_word(path, p >> 5) >> (p & 31)) & 1u;
        }
        // log q in free-bit order, as the batched scorer sums it
        lq += made_log_prob(T, bit);
        // every slot's bit for chain c: lane 16 s + c holds slot s's
        const uint64_t bits = __ballot(bit != 0u);
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const uint32_t bq = (uint32_t)(bits >> (16 * q + c)) & 1u;
            // the lattice bit at p is the free bit itself: flip its cone when
            // the new value differs from the current one
            const uint32_t m = 0u - (((pick_word(lat[q], p >> 5) >> (p & 31)) & 1u) ^ bq);
#pragma unroll
            for (int w = 0; w < NX; ++w) lat[q][w] ^= m & rec[8 + w];  // cone words, zero beyond W
        }
    }
    if (g < S && my_valid) {
        if (my_q == 0) {
            if (a.out && qs > 0) {
#pragma unroll
                for (int w = 0; w < NX; ++w) {
                    uint32_t v = 0u;
#pragma unroll
                    for (int q = 0; q < S; ++q) v = (q == my_s) ? lat[q][w] : v;
                    if (w < W) a.out[(int64_t)w * a.n + my_chain] = v;
                }
            }
            a.logq[my_chain] = lq;
        } else {
            a.logq_cur[my_chain] = lq;
        }
    }
}

// ---------------------------------------------------------------------------
// wide register-resident sampler (256 < H <= 1024, lattices of <= 512 bits,
// at most 128 free bits)
// ---------------------------------------------------------------------------
// The procedure of made_sample_reg_kernel for networks whose weights do not
// fit in LDS.  Each wave serves 16 chains and keeps in registers their
// first-layer activations (32 chunks of four dwords) and the logits of every
// free bit (8 blocks of 16 free bits, one MFMA accumulator each); the
// second-layer activations are never stored.  The network is streamed step
// by step.  A step is one half tile of a phase (16 hidden units): layer 1
// (weight rows of W1 against the chains' inputs) or layer 2 (rows of W2
// against the first-layer activations).  A layer-2 half tile's outputs that
// belong to the phase are final once computed, so their terms of every
// logit, V[p][u] a_u for the free positions p, are added to the logit
// accumulators right away (a 16 x 16 x 16 product per block of free bits,
// units outside the phase masked to zero so each unit is added once); V's
// mask makes the terms of positions that come before the unit's degree
// zero.  When a free bit is drawn its logit is therefore complete.  The four
// waves of a workgroup run the same steps: the 256 threads copy the next
// step's rows from global memory into one of two LDS buffers while every
// wave computes the current step from the other (rows whose K runs over
// hidden units stored in the k-slot order of stage_rows_k), and one barrier
// a step hands the buffers over.  64 chains are in flight per CU (one wave
// per SIMD), twice made_sample_kernel's 32.  Every activation is computed as
// the batched GEMMs compute it (one MFMA chain over the K chunks from zero,
// bias, ReLU, bf16), so the scorer of these networks is the GEMMs for both
// layers followed by wd_replay_kernel, which adds the logit terms in this
// kernel's order: sampler and scorer give the same log q bit for bit.
constexpr int WD_NH = 32;               // hidden chunks (H <= 1024)
constexpr int WD_NX = 16;               // lattice words = input chunks (<= 512 bits)
constexpr int WD_NB = 8;                // blocks of 16 free bits (h <= 128)
constexpr int WD_RS = 32 * WD_NH + 8;   // LDS row stride of a staged half tile (elements)
constexpr int WD_VS = 16;               // LDS row stride of a staged V block (elements)
constexpr int WD_BUF = 16 * WD_RS + 16 * WD_NB * WD_VS;  // elements of one step buffer
static_assert(2 * WD_BUF * 2 >= 16 * WD_NB * 64 * 8, "the log terms of a pass fit in the step buffers");

struct WdLayout {
    size_t lut, b1, b2, c, fp, rnd, buf, total;
};

__host__ __device__ inline WdLayout wd_layout(int D, int H) {
    WdLayout L;
    L.lut = 0;
    L.b1 = 256 * 16;
    L.b2 = L.b1 + (size_t)H * 4;
    L.c = L.b2 + (size_t)H * 4;
    L.fp = L.c + (size_t)D * 4;
    L.rnd = (L.fp + 16 * WD_NB * 4 + 15) & ~(size_t)15;
    L.buf = L.rnd + (size_t)16 * WD_NB * 64 * 4;
    L.total = L.buf + (size_t)2 * WD_BUF * 2;
    return L;
}

bool made_sample_wide_ok(const SampleArgs &a) {
    return a.H > 256 && a.H <= 32 * WD_NH && a.W <= WD_NX && a.DP <= 32 * WD_NX && a.h <= 16 * WD_NB &&
           wd_layout(a.D, a.H).total <= 160 * 1024;
}

// A staged step: thread t holds piece t (elements 4t .. 4t + 3) of the 16
// weight rows where the rows have it, and for a layer-2 step pieces t and
// t + 256 of the V block (free bit f = piece / 4, units 16 ht + 4 (piece % 4)
// .. + 3 of position fp[f]; voff[j] is the offset of piece t + 256 j in VT
// without the 16 ht, for f >= h that of an existing row).
struct WdStage {
    uint2 w[16];
    uint2 v[2];
};

__device__ __forceinline__ void wd_fetch(const SampleArgs &a, const uint32_t (&voff)[2], int4 st, WdStage &x) {
    const int t = threadIdx.x;
    const int np = 8 * st.z;  // pieces a row
    const bf16 *src = (st.x == 0 ? a.W1T + (int64_t)st.y * a.DP : a.W2T + (int64_t)st.y * a.H);
    const int64_t rs = st.x == 0 ? a.DP : a.H;
    if (t < np) {
#pragma unroll
        for (int r = 0; r < 16; ++r) x.w[r] = *reinterpret_cast<const uint2 *>(src + (int64_t)r * rs + 4 * t);
    }
    if (st.x == 1) {
#pragma unroll
        for (int j = 0; j < 2; ++j) x.v[j] = *reinterpret_cast<const uint2 *>(a.VT + voff[j] + st.y);
    }
}

// V pieces of free bits at or past h are stored as zeros.
__device__ __forceinline__ void wd_store(bf16 *buf, int4 st, const WdStage &x, int h) {
    const int t = threadIdx.x;
    const int np = 8 * st.z;
    // inputs keep their order; hidden units take the k-slot 8 g + 4 t' + e
    // of unit 16 t' + 4 g + e inside each 32-unit chunk
    const int slot = st.x == 0 ? 4 * t : 32 * (t >> 3) + 8 * (t & 3) + 4 * ((t >> 2) & 1);
    if (t < np) {
#pragma unroll
        for (int r = 0; r < 16; ++r) *reinterpret_cast<uint2 *>(buf + r * WD_RS + slot) = x.w[r];
    }
    if (st.x == 1) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int pc = t + 256 * j;
            *reinterpret_cast<uint2 *>(buf + 16 * WD_RS + (pc >> 2) * WD_VS + 4 * (pc & 3)) =
                (pc >> 2) < h ? x.v[j] : uint2{0u, 0u};
        }
    }
}

// A lane's first-layer activations: chunk k (hidden units 32 k .. 32 k + 31
// in k-slot order) is dwords 4 k .. 4 k + 3; vectors of 32 dwords, so that a
// write at a wave-uniform index is an indexed register move.
typedef uint32_t u32x32 __attribute__((ext_vector_type(32)));
typedef uint32_t u32x4w __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
struct WdAct {
    u32x32 q0, q1, q2, q3;
};
static_assert(WD_NH == 32, "four activation vectors");

__device__ __forceinline__ bf16x8 wd_chunk(const WdAct &a, int k) {
    const u32x32 &v = (k >> 3) == 0 ? a.q0 : ((k >> 3) == 1 ? a.q1 : ((k >> 3) == 2 ? a.q2 : a.q3));
    const int b = 4 * (k & 7);
    const u32x4w r = {v[b], v[b + 1], v[b + 2], v[b + 3]};
    return __builtin_bit_cast(bf16x8, r);
}

// half tile ht (units 16 ht + 4 g + e of the lane's chain) = dwords 2 ht, 2 ht + 1
__device__ __forceinline__ void wd_put(WdAct &a, int ht, uint32_t lo, uint32_t hi) {
    const int e = 2 * (ht & 15);
    switch (ht >> 4) {
    case 0:
        a.q0[e] = lo;
        a.q0[e + 1] = hi;
        break;
    case 1:
        a.q1[e] = lo;
        a.q1[e + 1] = hi;
        break;
    case 2:
        a.q2[e] = lo;
        a.q2[e + 1] = hi;
        break;
    default:
        a.q3[e] = lo;
        a.q3[e + 1] = hi;
        break;
    }
}

// One step on the staged rows `cur` (see made_sample_wide_kernel).  The K
// chunks run in groups of eight whose A (and layer-1 B) operands are read
// from LDS together; nk is a multiple of 8 except at the end of a row, so
// only a row's last group selects zero operands past nk.
__device__ __forceinline__ void wd_step(const bf16 *cur, int4 st, int c, int g, const uint32_t (&lat)[WD_NX],
                                        WdAct &act1, f32x4 (&lacc)[WD_NB], const bf16x8 *lut, const float *b1s,
                                        const float *b2s) {
    const int nk = st.z, ht = st.y >> 4;
    // units 16 ht + r (A row r = c) against the lane's chain: outputs unit
    // 16 ht + 4 g + e of chain c
    const bf16 *arow = cur + c * WD_RS + 8 * g;
    const bf16x8 zero = {};
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if (st.x == 0) {
#pragma unroll
        for (int q = 0; q < WD_NX / 8; ++q) {
            if (8 * q >= nk) break;
            bf16x8 av[8], bv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                av[j] = *reinterpret_cast<const bf16x8 *>(arow + 32 * (8 * q + j));
                bv[j] = lut[(lat[8 * q + j] >> (8 * g)) & 0xffu];
            }
            if (8 * q + 8 <= nk) {
#pragma unroll
                for (int j = 0; j < 8; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[j], bv[j], acc, 0, 0, 0);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(8 * q + j < nk ? av[j] : zero, bv[j], acc, 0, 0, 0);
            }
        }
        const float *bias = b1s + st.y + 4 * g;
        wd_put(act1, ht, pack_bf16(relu(acc[0] + bias[0]), relu(acc[1] + bias[1])),
               pack_bf16(relu(acc[2] + bias[2]), relu(acc[3] + bias[3])));
    } else {
#pragma unroll
        for (int q = 0; q < WD_NH / 8; ++q) {
            if (8 * q >= nk) break;
            bf16x8 av[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) av[j] = *reinterpret_cast<const bf16x8 *>(arow + 32 * (8 * q + j));
            if (8 * q + 8 <= nk) {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[j], wd_chunk(act1, 8 * q + j), acc, 0, 0, 0);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(8 * q + j < nk ? av[j] : zero,
                                                                  wd_chunk(act1, 8 * q + j), acc, 0, 0, 0);
            }
        }
        // the phase's units of the half tile, as the B operand (K = unit
        // 16 ht + 4 g + e) of the logit blocks' products
        const int lo = st.w & 0xff, hi = st.w >> 8;
        const float *bias = b2s + st.y + 4 * g;
        float y[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int u = 4 * g + e;
            y[e] = (u >= lo && u < hi) ? relu(acc[e] + bias[e]) : 0.f;
        }
        const s16x4 bv = __builtin_bit_cast(s16x4, uint2{pack_bf16(y[0], y[1]), pack_bf16(y[2], y[3])});
        const bf16 *vrow = cur + 16 * WD_RS + c * WD_VS + 4 * g;
        s16x4 va[WD_NB];
#pragma unroll
        for (int b = 0; b < WD_NB; ++b) va[b] = *reinterpret_cast<const s16x4 *>(vrow + 16 * b * WD_VS);
#pragma unroll
        for (int b = 0; b < WD_NB; ++b) lacc[b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(va[b], bv, lacc[b], 0, 0, 0);
    }
}

// The schedule and the cones are read-only for the whole launch and read at
// wave-uniform addresses: through the constant address space they become
// scalar loads, batched where consecutive.
typedef const __attribute__((address_space(4))) int *wd_cint;
typedef const __attribute__((address_space(4))) uint32_t *wd_cu32;

__device__ __forceinline__ int4 wd_sched(wd_cint p, int i) {
    return int4{p[4 * i], p[4 * i + 1], p[4 * i + 2], p[4 * i + 3]};
}

__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1))) void
made_sample_wide_kernel(SampleArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const WdLayout L = wd_layout(a.D, a.H);
    bf16x8 *lut = reinterpret_cast<bf16x8 *>(smem + L.lut);
    float *b1s = reinterpret_cast<float *>(smem + L.b1);
    float *b2s = reinterpret_cast<float *>(smem + L.b2);
    float *cs = reinterpret_cast<float *>(smem + L.c);
    int *fp = reinterpret_cast<int *>(smem + L.fp);
    // [free bit][chain of the workgroup]: the Philox word of the draw, then
    // the probability word of the chosen bit (see below)
    uint32_t *rnd = reinterpret_cast<uint32_t *>(smem + L.rnd);
    bf16 *buf = reinterpret_cast<bf16 *>(smem + L.buf);
    for (int i = threadIdx.x; i < 256; i += blockDim.x) lut[i] = bits_to_bf16x8((uint32_t)i);
    for (int i = threadIdx.x; i < a.H; i += blockDim.x) {
        b1s[i] = a.b1[i];
        b2s[i] = a.b2[i];
    }
    for (int i = threadIdx.x; i < a.D; i += blockDim.x) cs[i] = a.c[i];
    for (int i = threadIdx.x; i < a.h; i += blockDim.x) fp[i] = a.wphase[i].z;
    __syncthreads();
    const wd_cint wph = (wd_cint)(const int *)a.wphase, wst = (wd_cint)(const int *)a.wstep;
    const wd_cu32 wcn = (wd_cu32)a.wcone;

    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    const int wave = threadIdx.x >> 6;
    const int wc = 16 * wave + c;  // the chain's column of rnd
    const int my_chain = (blockIdx.x * 4 + wave) * 16 + c;
    const bool valid = my_chain < a.n;
    const uint32_t *B = a.blob;
    const uint32_t *cw = B + B[H_OFF_CONST];
    const uint32_t cid = B[H_CID];
    const int W = a.W;
    // the chain's Philox words of the whole pass (one call per four free
    // bits), computed up front with the calls spread over its four lane
    // groups instead of one dependent call every fourth draw
    if (!a.score) {
        for (int i = g; 4 * i < a.h; i += 4) {
            const U4 u4 = philox4x32_10(a.step, (uint32_t)i, a.chain_begin + (uint32_t)my_chain, cid | (1u << 16),
                                        a.seed_lo, a.seed_hi);
            rnd[(4 * i + 0) * 64 + wc] = u4.x;
            rnd[(4 * i + 1) * 64 + wc] = u4.y;
            rnd[(4 * i + 2) * 64 + wc] = u4.z;
            rnd[(4 * i + 3) * 64 + wc] = u4.w;
        }
    }

    uint32_t lat[WD_NX];
    WdAct act1;
    f32x4 lacc[WD_NB];
#pragma unroll
    for (int w = 0; w < WD_NX; ++w) lat[w] = w < W ? cw[w] : 0u;
    act1.q0 = act1.q1 = act1.q2 = act1.q3 = u32x32{};
#pragma unroll
    for (int b = 0; b < WD_NB; ++b) lacc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    WdStage x;
    // The phases' steps are consecutive from step 0.  The schedule records
    // are read one step (one phase) ahead of their use, so that their
    // scalar loads are in flight while a step computes: st is the record of
    // step sidx, s_next that of step sidx + 1, ph_next that of the next phase.
    const int4 zero4 = {0, 0, 0, 0};
    int4 st = a.nsteps > 0 ? wd_sched(wst, 0) : zero4;
    int4 s_next = a.nsteps > 1 ? wd_sched(wst, 1) : zero4;
    int4 ph_next = a.h > 0 ? wd_sched(wph, 0) : zero4;
    uint32_t voff[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int pc = threadIdx.x + 256 * j, f = min(pc >> 2, max(a.h - 1, 0));
        voff[j] = (uint32_t)(a.h > 0 ? fp[f] : 0) * (uint32_t)a.H + 4u * (uint32_t)(pc & 3);
    }
    if (a.nsteps > 0) {
        wd_fetch(a, voff, st, x);
        wd_store(buf, st, x, a.h);
    }
    __syncthreads();
    int sidx = 0;
    for (int f = 0; f < a.h; ++f) {
        const int4 ph = ph_next;  // {first step, end step, p, 0}
        if (f + 1 < a.h) ph_next = wd_sched(wph, f + 1);
        const int p = ph.z;
        // the cone of free bit f (16 words, zero past W), loaded now and
        // applied after the phase's steps
        uint32_t cone[WD_NX];
#pragma unroll
        for (int w = 0; w < WD_NX; ++w) cone[w] = wcn[(size_t)f * a.cone_stride + w];
        // score mode: the scored path's word holding bit p, loaded now and
        // used after the phase's steps
        const uint32_t pw = (a.score && valid) ? a.score[(int64_t)(p >> 5) * a.n + my_chain] : 0u;
        for (; sidx < ph.y; ++sidx) {
            // {layer (0, 1), first unit 16 ht, K chunks, units of the phase
            // in the half tile: [lo, hi) as lo | hi << 8}
            const bf16 *cur = buf + (sidx & 1) * WD_BUF;
            const bool more = sidx + 1 < a.nsteps;
            const int4 nx = s_next;
            if (sidx + 2 < a.nsteps) s_next = wd_sched(wst, sidx + 2);
            if (more) wd_fetch(a, voff, nx, x);  // in flight during this step's products
            wd_step(cur, st, c, g, lat, act1, lacc, lut, b1s, b2s);
            if (more) wd_store(buf + ((sidx + 1) & 1) * WD_BUF, nx, x, a.h);
            __syncthreads();
            st = nx;
        }
        // the logit of free bit f: element f & 3 of block f >> 4 on the lanes
        // of group (f & 15) >> 2, passed to the chain's four lane groups
        float mine = 0.f;
#pragma unroll
        for (int b = 0; b < WD_NB; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if ((f >> 4) == b && (f & 3) == e) mine = lacc[b][e];
        const float lg = __shfl(mine, c + 16 * ((f & 15) >> 2), 64);
        // the bit of free bit f: drawn against the threshold of the logit,
        // or read from the scored path; every lane group does its chain's
        const uint32_t T = made_threshold(lg + cs[p]);
        const uint32_t bit = !a.score ? (rnd[f * 64 + wc] < T ? 1u : 0u) : (pw >> (p & 31)) & 1u;
        // the bit's probability times 2^32, T for a 1 and 2^32 - T for a 0
        // (both in [1, 2^32 - 1]); its logarithm is taken after the pass
        if (g == 0) rnd[f * 64 + wc] = bit ? T : 0u - T;
        // the lattice bit at p is the free bit itself: flip its cone when
        // the new value differs from the current one
        const uint32_t m = 0u - (((pick_word(lat, p >> 5) >> (p & 31)) & 1u) ^ bit);
#pragma unroll
        for (int w = 0; w < WD_NX; ++w) lat[w] ^= m & cone[w];
    }
    // log q: the logarithms of the probability words, spread over the
    // chain's lane groups (the step buffers are free now), then added in
    // free-bit order by one lane, as made_log_prob terms are added everywhere
    __syncthreads();
    double *lt = reinterpret_cast<double *>(buf);  // [free bit][chain of the workgroup]
    for (int f = g; f < a.h; f += 4) lt[f * 64 + wc] = made_log((double)rnd[f * 64 + wc] * 0x1p-32);
    __syncthreads();
    if (g == 0 && valid) {
        double lq = 0.0;
        for (int f = 0; f < a.h; ++f) lq += lt[f * 64 + wc];
        if (a.out && !a.score)
            for (int w = 0; w < W; ++w) a.out[(int64_t)w * a.n + my_chain] = pick_word(lat, w);
        a.logq[my_chain] = lq;
    }
}

hipError_t launch_wide(const SampleArgs &a, hipStream_t s) {
    const size_t lds = wd_layout(a.D, a.H).total;
    const int grid = (a.n + 63) / 64;
    if (a.cone_stride < WD_NX) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)made_sample_wide_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(made_sample_wide_kernel, dim3(grid), dim3(256), lds, s, a);
    return hipGetLastError();
}

// The scorer's last stage for the networks of made_sample_wide_kernel: the
// logits of the scored paths from their second-layer activations H2 (the
// GEMMs' bf16 output, row per path), added in the sampler's order (each
// layer-2 step in turn: the phase's units of the half tile against the rows
// of V of every free bit, one 16 x 16 x 16 product per block of 16 free
// bits), and log q as the sampler sums it.  The sampler reads the logit of a
// free bit after the steps of its phase; the later steps add to it only
// products with weights V's mask keeps at zero (+0 each), so reading every
// logit after the last step gives the same bits.
// A workgroup scores 64 paths, a wave 16 of them (lane (c, g): path c,
// units 4 g .. 4 g + 3 of a half tile) over all blocks.  The steps come in
// 64-unit panels (the step list's half tiles never decrease): the panel's
// columns of V for every free bit and of H2 for the 64 paths are staged in
// LDS with whole-row loads, the next panel's loads in flight while the
// current one's steps run.
constexpr int WD_MAXL2 = 2 * WD_NH + 2 * 16 * WD_NB;  // layer-2 steps of a schedule, at most
constexpr int RP_PS = 64 + 4;                          // LDS row stride of a panel (elements)
constexpr int RP_V = 16 * WD_NB * RP_PS;               // elements of a V panel
constexpr int RP_H = 64 * RP_PS;                       // elements of an H2 panel
constexpr int RP_STAGE = (RP_V + RP_H) * 2;            // bytes of one stage
constexpr int RP_LC = 32;                              // free bits of a chunk of log q terms
constexpr int RP_END = 16 * WD_NB * 64 * 4 + RP_LC * 64 * 8;  // bytes of the logits and log q terms

__global__ __launch_bounds__(256) void wd_replay_kernel(ReplayArgs a) {
    __shared__ __align__(16) unsigned char sm[2 * RP_STAGE > RP_END ? 2 * RP_STAGE : RP_END];
    __shared__ int2 l2s[WD_MAXL2];
    __shared__ int fps[16 * WD_NB];
    for (int i = threadIdx.x; i < a.n2; i += blockDim.x) l2s[i] = a.l2[i];
    for (int i = threadIdx.x; i < 16 * WD_NB; i += blockDim.x) fps[i] = i < a.h ? a.fpos[i] : 0;
    __syncthreads();
    const int t = threadIdx.x, lane = t & 63, c = lane & 15, g = lane >> 4, wave = t >> 6;
    const int pbase = blockIdx.x * 64;  // first path of the workgroup in the batch
    // panel k's pieces of 16 bytes: V row f = i >> 3 (the row of free bit f,
    // zero past the last), H2 row r (path pbase + r, clamped)
    uint4 pv[4], ph[2];
    auto fetch = [&](int k) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int id = t + 256 * i, f = id >> 3;
            pv[i] = *reinterpret_cast<const uint4 *>(a.VT + (int64_t)fps[f] * a.H + 64 * k + 8 * (id & 7));
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int id = t + 256 * i, r = id >> 3, j = pbase + r < a.nb ? pbase + r : 0;
            ph[i] = *reinterpret_cast<const uint4 *>(a.H2 + (int64_t)j * a.H + 64 * k + 8 * (id & 7));
        }
    };
    auto stage = [&](int buf) __attribute__((always_inline)) {
        bf16 *V = reinterpret_cast<bf16 *>(sm + buf * RP_STAGE), *Hs = V + RP_V;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int id = t + 256 * i, f = id >> 3;
            *reinterpret_cast<uint4 *>(V + f * RP_PS + 8 * (id & 7)) = f < a.h ? pv[i] : uint4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int id = t + 256 * i;
            *reinterpret_cast<uint4 *>(Hs + (id >> 3) * RP_PS + 8 * (id & 7)) = ph[i];
        }
    };
    f32x4 lacc[WD_NB];
#pragma unroll
    for (int b = 0; b < WD_NB; ++b) lacc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int np = a.H / 64;
    fetch(0);
    stage(0);
    __syncthreads();
    int si = 0;
    for (int k = 0; k < np; ++k) {
        if (k + 1 < np) fetch(k + 1);
        const bf16 *V = reinterpret_cast<const bf16 *>(sm + (k & 1) * RP_STAGE), *Hs = V + RP_V;
        for (; si < a.n2 && (l2s[si].x >> 6) == k; ++si) {
            const int2 st = l2s[si];
            const int lo = st.y & 0xff, hi = (st.y >> 8) & 0xff, u0 = (st.x & 63) + 4 * g;
            uint2 h = *reinterpret_cast<const uint2 *>(Hs + (16 * wave + c) * RP_PS + u0);
            // units of the half tile outside the phase: zero
            const int v0 = 4 * g;
            if (!(v0 >= lo && v0 < hi)) h.x &= 0xffff0000u;
            if (!(v0 + 1 >= lo && v0 + 1 < hi)) h.x &= 0x0000ffffu;
            if (!(v0 + 2 >= lo && v0 + 2 < hi)) h.y &= 0xffff0000u;
            if (!(v0 + 3 >= lo && v0 + 3 < hi)) h.y &= 0x0000ffffu;
            const s16x4 bv = __builtin_bit_cast(s16x4, h);
            s16x4 va[WD_NB];
#pragma unroll
            for (int b = 0; b < WD_NB; ++b)
                va[b] = *reinterpret_cast<const s16x4 *>(V + (16 * b + c) * RP_PS + u0);
#pragma unroll
            for (int b = 0; b < WD_NB; ++b)
                lacc[b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(va[b], bv, lacc[b], 0, 0, 0);
        }
        __syncthreads();
        if (k + 1 < np) stage((k + 1) & 1);
        __syncthreads();
    }
    // lane (c, g) holds free bits 16 b + 4 g + e of path 16 wave + c; the
    // stages' LDS now takes the logits and the log q terms
    float *lgt = reinterpret_cast<float *>(sm);                         // [free bit][path]
    double *lp = reinterpret_cast<double *>(sm + 16 * WD_NB * 64 * 4);  // [free bit of the chunk][path]
#pragma unroll
    for (int b = 0; b < WD_NB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) lgt[(16 * b + 4 * g + e) * 64 + 16 * wave + c] = lacc[b][e];
    __syncthreads();
    // the log q terms of RP_LC free bits at a time in parallel, then each
    // path adds them to its sum in free-bit order
    double lq = 0.0;
    for (int f0 = 0; f0 < a.h; f0 += RP_LC) {
        for (int idx = t; idx < 64 * RP_LC; idx += blockDim.x) {
            const int f = f0 + (idx >> 6), r = idx & 63, j = pbase + r;
            if (f < a.h && j < a.nb) {
                const int p = fps[f];
                const uint32_t T = made_threshold(lgt[f * 64 + r] + a.c[p]);
                const uint32_t w = a.states[(int64_t)(p >> 5) * a.n + a.b0 + j];
                lp[idx] = made_log_prob(T, (w >> (p & 31)) & 1u);
            }
        }
        __syncthreads();
        if (t < 64) {
            const int fe = f0 + RP_LC < a.h ? f0 + RP_LC : a.h;
            for (int f = f0; f < fe; ++f) lq += lp[(f - f0) * 64 + t];
        }
        __syncthreads();
    }
    if (t < 64 && pbase + t < a.nb) a.logq[pbase + t] = lq;
}

hipError_t launch_wide_replay(const ReplayArgs &a, hipStream_t s) {
    if (a.nb <= 0) return hipSuccess;
    if (a.h > 16 * WD_NB || a.H % 64 || a.n2 < 0 || a.n2 > WD_MAXL2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wd_replay_kernel, dim3((a.nb + 63) / 64), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int NX, int NH, int NB, int NP, bool FULL>
hipError_t launch_reg_k(const SampleArgs &a, size_t lds, hipStream_t s) {
    // enough waves per workgroup to share the staged network, few enough to
    // spread small runs over every CU
    const int waves = (a.n + 16 * NB - 1) / (16 * NB);
    const int per_wg = std::min(8, std::max(1, waves / 512));
    const int grid = (waves + per_wg - 1) / per_wg;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)made_sample_reg_kernel<NX, NH, NB, NP, FULL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((made_sample_reg_kernel<NX, NH, NB, NP, FULL>), dim3(grid), dim3(64 * per_wg), lds, s, a);
    return hipGetLastError();
}

// chain blocks per wave: four slots (one chain-path per lane) where the
// activations and lattices of four slots fit in registers without spilling,
// fewer for wider networks or lattices
template <int NX, int NH, int NP>
constexpr int reg_blocks() {
    if (NH <= 2) return 4 / NP;
    if (NH <= 4) return NX <= 2 ? 4 / NP : (NP == 1 ? 2 : 1);
    return 1;
}

// Rows of exactly 2, 4 or 8 chunks take the full-chunk kernel (sized for
// them); any other shape within the limits takes one guarded kernel sized for
// the largest (8 and 8 chunks, one slot), which keeps the number of kernels
// compiled small.
int reg_chunks(int len) { return len == 64 ? 2 : (len == 128 ? 4 : (len == 256 ? 8 : 0)); }

template <int NX, int NH, int NP>
hipError_t launch_full(const SampleArgs &a, size_t lds, hipStream_t s) {
    return launch_reg_k<NX, NH, reg_blocks<NX, NH, NP>(), NP, true>(a, lds, s);
}

template <int NX, int NP>
hipError_t launch_full_h(const SampleArgs &a, size_t lds, hipStream_t s) {
    if (reg_chunks(a.H) == 2) return launch_full<NX, 2, NP>(a, lds, s);
    return launch_full<NX, 4, NP>(a, lds, s);  // H = 128 (a 256-wide network does not fit in LDS)
}

template <int NP>
hipError_t launch_full_w(const SampleArgs &a, size_t lds, hipStream_t s) {
    const int nx = reg_chunks(a.DP);
    if (nx == 2) return launch_full_h<2, NP>(a, lds, s);
    if (nx == 4) return launch_full_h<4, NP>(a, lds, s);
    return launch_full_h<(NP == 1 ? 8 : 4), NP>(a, lds, s);  // dual: W <= 4
}

bool reg_fits(const SampleArgs &a) {
    return a.H <= 256 && a.W <= 8 && reg_layout(a.D, a.DP, a.H).total <= 160 * 1024;
}

bool made_sample_dual_ok(const SampleArgs &a) {
    // two paths of 256-wide activations, or of 8-word lattices beside 128-wide
    // ones, would not fit in registers; other shapes than whole rows of 2 or 4
    // chunks run the two calls
    const int nx = reg_chunks(a.DP), nh = reg_chunks(a.H);
    return reg_fits(a) && (nx == 2 || nx == 4) && (nh == 2 || nh == 4);
}

hipError_t launch_made_sample_dual(const SampleArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    return launch_full_w<2>(a, reg_layout(a.D, a.DP, a.H).total, s);
}

// LDS of made_sample_kernel for the shape in a; sets a.defer (small networks
// defer the log-probabilities to the end and keep the cones in LDS; the log
// buffer reuses the activations when they are large enough)
static size_t made_sample_lds(SampleArgs &a) {
    const size_t base = (size_t)16 * (a.DP + 8) * 2 + (size_t)2 * 16 * (a.H + 8) * 2 + 16 * 4 + (size_t)16 * a.W * 4;
    a.defer = 0;
    size_t lds = base;
    if (a.H <= 256) {
        const size_t ts = (size_t)a.h * 16 * 4, cn = (size_t)((a.h * a.W + 1) & ~1) * 4;
        const size_t lg = (size_t)a.h * 16 * 8;
        a.defer = lg <= (size_t)2 * 16 * a.H * 2 ? 2 : 1;
        lds = base + ts + cn + (a.defer == 1 ? lg : 0);
    }
    return lds;
}

bool made_sample_launchable(const SampleArgs &a0) {
    SampleArgs a = a0;
    return reg_fits(a) || made_sample_wide_ok(a) || made_sample_lds(a) <= 160 * 1024;
}

hipError_t launch_made_sample(const SampleArgs &a0, hipStream_t s) {
    SampleArgs a = a0;
    if (a.n <= 0) return hipSuccess;
    // small networks and lattices: the register-resident kernel
    if (reg_fits(a)) {
        const size_t lds = reg_layout(a.D, a.DP, a.H).total;
        if (reg_chunks(a.DP) && (a.H == 64 || a.H == 128)) return launch_full_w<1>(a, lds, s);
        return launch_reg_k<8, 8, 1, 1, false>(a, lds, s);
    }
    // wider networks on lattices of at most 512 bits: the wide one
    if (made_sample_wide_ok(a) && a.wstep) return launch_wide(a, s);
    const int grid = (a.n + 15) / 16;
    const size_t lds = made_sample_lds(a);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)made_sample_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(made_sample_kernel, dim3(grid), dim3(64), lds, s, a);
    return hipGetLastError();
}

__global__ void log_eval_kernel(const double *__restrict__ x, double *__restrict__ y, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = made_log(x[i]);
}

hipError_t launch_log_eval(const double *x, double *y, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(log_eval_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t launch_unpack(const uint32_t *states, int n, int D, int DP, bf16 *X, hipStream_t s) {
    const int64_t tot = (int64_t)n * DP;
    hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, states, n, D, DP, X);
    return hipGetLastError();
}

hipError_t launch_gate_colsum(bf16 *G, const bf16 *A, int n, int N, float *colpart, hipStream_t s) {
    if (n <= 0 || N <= 0) return hipSuccess;
    if (N % 8 || (((uintptr_t)G) & 15) || (((uintptr_t)A) & 15)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gate_colsum_kernel, dim3((unsigned)((N + 127) / 128), (unsigned)((n + 63) / 64)), dim3(256), 0,
                       s, G, A, n, N, colpart);
    return hipGetLastError();
}

hipError_t launch_grad_final(const GradFinal &a, hipStream_t s) {
    if (a.P <= 0) return hipSuccess;
    if (a.zW1 < 1 || a.zW2 < 1 || a.zV < 1 || a.chunks < 1 || (a.adam && (!a.th || !a.m || !a.v)) ||
        (!a.adam && !a.grad))
        return hipErrorInvalidValue;
    if (a.adam && a.sh[0].Wb) {
        // the three weights' shapes and offsets must be the flat layout's
        const int64_t D = a.D, H = a.H;
        const ShadowJob *J = a.sh;
        const bool shapes = J[0].K == a.D && J[0].N == a.H && J[1].K == a.H && J[1].N == a.H && J[2].K == a.H &&
                            J[2].N == a.D && a.ob1 == a.oW1 + D * H && a.ob2 == a.oW2 + H * H &&
                            a.oc == a.oV + H * D && a.oW2 == a.ob1 + H && a.oV == a.ob2 + H && a.P == a.oc + D;
        int tc[3];
        int64_t blocks = 0;
        for (int w = 0; w < 3; ++w) {
            if (!J[w].Wb || !J[w].WT || J[w].KP < J[w].K || J[w].K <= 0 || J[w].N <= 0) return hipErrorInvalidValue;
            tc[w] = ((J[w].N + AS_COLS - 1) / AS_COLS) * ((J[w].KP + AS_ROWS - 1) / AS_ROWS);
            blocks += tc[w];
        }
        if (!shapes) return hipErrorInvalidValue;
        blocks += (2 * H + D + 255) / 256;
        if (a.ux_n > 0) {
            const int64_t ue = (int64_t)a.ux_n * (a.ux_DP / 8);
            if (!a.ux_states || !a.ux_X || a.ux_DP % 32 || a.ux_DP < a.D || ue > (int64_t)UINT32_MAX)
                return hipErrorInvalidValue;
            blocks += (ue + 255) / 256;
        }
        if (blocks > INT32_MAX) return hipErrorInvalidValue;
        hipLaunchKernelGGL(adam_shadow_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, int4{tc[0], tc[1], tc[2], 0});
        return hipGetLastError();
    }
    hipLaunchKernelGGL(grad_final_kernel, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_shadow(const ShadowJobs &jobs, int count, hipStream_t s) {
    if (count < 1 || count > 3) return hipErrorInvalidValue;
    int gx = 0, gy = 0;
    for (int i = 0; i < count; ++i) {
        gx = std::max(gx, (jobs.j[i].N + 31) / 32);
        gy = std::max(gy, (jobs.j[i].KP + 31) / 32);
    }
    if (gx == 0 || gy == 0) return hipSuccess;
    hipLaunchKernelGGL(shadow_kernel, dim3(gx, gy, count), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_logq(const float *L, const uint32_t *states, uint64_t stride, uint64_t b0, const int *fpos, int h,
                       int n, int D, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(logq_kernel, dim3((n + 63) / 64), dim3(256), 0, s, L, states, stride, b0, fpos, h, n, D, out);
    return hipGetLastError();
}

}  // namespace pbit
