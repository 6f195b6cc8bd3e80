// Library GEMMs (hipBLASLt) for the activation products of a MADE training
// step (internal).  A training step's activations need not match the
// samplers' bits (the scorer's products, which must, stay on gemm_kernel),
// so the plain products run on the library's tuned kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "made.h"

namespace pbit {

struct LtState;

// A handle for the current device, or nullptr when the library cannot make
// one (the caller then keeps its own kernels).
LtState *lt_create();
void lt_destroy(LtState *lt);

// C[m][n] = act(sum_k A[m][k] W[n][k] + bias[n]) for row-major bf16 A (M x K,
// row stride lda), W (N x K, ldw) and C (M x N, ldc); bias (fp32, N) may be
// NULL; act is ReLU or the identity; FP32 accumulation, C rounded to bf16.
// Algorithms are chosen once per shape by the library's heuristic and kept,
// so a shape always runs the same kernel.  Returns false when the library has
// no algorithm for the shape or a call fails (nothing was launched then, or
// the launch failed); `ws` (ws_bytes) is the library's workspace.
bool lt_gemm_nt(LtState *lt, int M, int N, int K, const bf16 *A, int64_t lda, const bf16 *W, int64_t ldw,
                const float *bias, bool relu, bf16 *C, int64_t ldc, void *ws, size_t ws_bytes, hipStream_t s);

// Workspace the products may use.
constexpr size_t LT_WORKSPACE = (size_t)32 << 20;

}  // namespace pbit
