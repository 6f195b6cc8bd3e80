// Learned proposal (MADE) and Metropolis-Hastings: internal interfaces.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/pbit.h"

namespace pbit {

typedef __bf16 bf16;

// One masked bf16 MFMA GEMM: C(m, n) = epilogue(sum_k A(m, k) B(k, n)).
// Strided operands (A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn])
// so transposed products need no copies.  The reduction of output column
// tile nt (64 columns) runs over [kbeg[nt], kend[nt]) in ascending 32-wide
// chunks, so every output is a fixed sequence of v_mfma_f32_16x16x32_bf16
// accumulations.  Products that feed
// the sampler's arithmetic never split K; the weight gradients may
// (ksplit slices summed in a fixed order by a second kernel).
struct GemmArgs {
    const bf16 *A;
    int64_t sam, sak;
    const bf16 *B;
    int64_t sbk, sbn;
    void *C;
    int64_t scm, scn;
    int M, N, K;
    const int *kbeg, *kend;  // per 64-column tile, may be NULL
    const float *bias;       // per column, may be NULL
    int relu;
    const bf16 *gate;        // multiply by (gate(m, n) > 0), may be NULL
    int64_t sgm, sgn;
    const int *deg_row, *deg_col;  // keep C(m, n) iff deg_row[m] <= deg_col[n]; may be NULL
    int out_bf16;
    int accumulate;          // fp32 output: C += result
    int ksplit;              // > 1: K split in that many slices (fp32 out, no bias / relu / gate)
    float *part;             // split-K workspace, ksplit x M x N floats
    // K runs over hidden units and both operands take the k-slot order of the
    // samplers inside each 32-wide chunk (k-slot 8 g + 4 t + e holds unit
    // 16 t + 4 g + e), so each output sums its products as the wide sampler
    // does; needs both operands in mode 0 (k contiguous)
    int kperm;
    // split-K partial sums stay in `part` (ksplit slices, or one with
    // ksplit <= 1) for a later reduction; no epilogue
    int keep_parts;
    // per 64-row tile column sums of the stored output, in a fixed order:
    // colpart[(m / 64) N + n] (fp32; bf16 outputs are summed as stored)
    float *colpart;
    // logits to loss gradient: C(m, n) becomes (sigmoid(v) - x) inv_n on the
    // columns with lossfree[n] (0 elsewhere), x = lossx[m slx + n], and each
    // tile's share of the batch-mean binary cross-entropy goes to
    // losspart[tile] (tiles numbered row-major over the 64 x 64 grid)
    const bf16 *lossx;
    int64_t slx;
    const int *lossfree;
    float inv_n;
    float *losspart;
};

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);

// Up to GEMM_GROUP_MAX split-K products whose slices stay for a later
// finalize (keep_parts, no epilogue), with one operand layout, in a single
// launch: their workgroups share the machine and one tail (products of
// different layouts get a launch each).  The slices are those launch_gemm
// would write, bit for bit.
constexpr int GEMM_GROUP_MAX = 3;
struct GemmGroup {
    GemmArgs g[GEMM_GROUP_MAX];
    int bx[GEMM_GROUP_MAX], z[GEMM_GROUP_MAX];  // blocks of a tile order (multiple of 8), slices
    int count;
};
hipError_t launch_gemm_group(const GemmArgs *gs, int count, hipStream_t s);

}  // namespace pbit
