// hipBLASLt products for the MADE training step; see blaslt.h.
#include "blaslt.h"

#include <hipblaslt/hipblaslt.h>

#include <deque>
#include <mutex>

namespace pbit {

namespace {

struct LtPlan {
    int M, N, K;
    int64_t lda, ldw, ldc;
    bool bias, relu;
    hipblasLtMatmulDesc_t desc = nullptr;
    hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, lc = nullptr;
    hipblasLtMatmulAlgo_t algo;
    size_t ws = 0;
    bool ok = false;
};

}  // namespace

struct LtState {
    hipblasLtHandle_t h = nullptr;
    std::mutex mu;
    std::deque<LtPlan> plans;  // stable addresses
    ~LtState() {
        for (auto &p : plans) {
            if (p.la) hipblasLtMatrixLayoutDestroy(p.la);
            if (p.lb) hipblasLtMatrixLayoutDestroy(p.lb);
            if (p.lc) hipblasLtMatrixLayoutDestroy(p.lc);
            if (p.desc) hipblasLtMatmulDescDestroy(p.desc);
        }
        if (h) hipblasLtDestroy(h);
    }
};

LtState *lt_create() {
    auto *lt = new LtState();
    if (hipblasLtCreate(&lt->h) != HIPBLAS_STATUS_SUCCESS) {
        lt->h = nullptr;
        delete lt;
        return nullptr;
    }
    return lt;
}

void lt_destroy(LtState *lt) { delete lt; }

namespace {

constexpr int LT_CANDIDATES = 8;

// The product in the library's column-major terms: C^T (N x M, ldc) =
// op(W) (N x K) op(A) (K x M), W stored K x N (ldw) and transposed, A stored
// K x M (lda); the bias runs along C^T's rows.  Fills res with the
// heuristic's candidates (got of them).
bool plan(LtState *lt, LtPlan &p, size_t ws_bytes, hipblasLtMatmulHeuristicResult_t *res, int &got) {
    const hipDataType bf = HIP_R_16BF;
    if (hipblasLtMatmulDescCreate(&p.desc, HIPBLAS_COMPUTE_32F, HIP_R_32F) != HIPBLAS_STATUS_SUCCESS) return false;
    const int32_t ta = HIPBLAS_OP_T, tb = HIPBLAS_OP_N;
    if (hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_TRANSA, &ta, sizeof(ta)) !=
            HIPBLAS_STATUS_SUCCESS ||
        hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_TRANSB, &tb, sizeof(tb)) !=
            HIPBLAS_STATUS_SUCCESS)
        return false;
    const uint32_t epi = p.bias ? (p.relu ? HIPBLASLT_EPILOGUE_RELU_BIAS : HIPBLASLT_EPILOGUE_BIAS)
                                : (p.relu ? HIPBLASLT_EPILOGUE_RELU : HIPBLASLT_EPILOGUE_DEFAULT);
    if (hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_EPILOGUE, &epi, sizeof(epi)) !=
        HIPBLAS_STATUS_SUCCESS)
        return false;
    if (p.bias) {
        const int32_t bt = HIP_R_32F;
        if (hipblasLtMatmulDescSetAttribute(p.desc, HIPBLASLT_MATMUL_DESC_BIAS_DATA_TYPE, &bt, sizeof(bt)) !=
            HIPBLAS_STATUS_SUCCESS)
            return false;
    }
    if (hipblasLtMatrixLayoutCreate(&p.la, bf, p.K, p.N, p.ldw) != HIPBLAS_STATUS_SUCCESS ||
        hipblasLtMatrixLayoutCreate(&p.lb, bf, p.K, p.M, p.lda) != HIPBLAS_STATUS_SUCCESS ||
        hipblasLtMatrixLayoutCreate(&p.lc, bf, p.N, p.M, p.ldc) != HIPBLAS_STATUS_SUCCESS)
        return false;
    hipblasLtMatmulPreference_t pref = nullptr;
    if (hipblasLtMatmulPreferenceCreate(&pref) != HIPBLAS_STATUS_SUCCESS) return false;
    const uint64_t wsz = ws_bytes;
    got = 0;
    const bool found =
        hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wsz, sizeof(wsz)) ==
            HIPBLAS_STATUS_SUCCESS &&
        hipblasLtMatmulAlgoGetHeuristic(lt->h, p.desc, p.la, p.lb, p.lc, p.lc, pref, LT_CANDIDATES, res, &got) ==
            HIPBLAS_STATUS_SUCCESS;
    hipblasLtMatmulPreferenceDestroy(pref);
    if (!found) got = 0;
    int kept = 0;
    for (int i = 0; i < got; ++i)
        if (res[i].state == HIPBLAS_STATUS_SUCCESS && res[i].workspaceSize <= ws_bytes) res[kept++] = res[i];
    got = kept;
    return got > 0;
}

}  // namespace

bool lt_gemm_nt(LtState *lt, int M, int N, int K, const bf16 *A, int64_t lda, const bf16 *W, int64_t ldw,
                const float *bias, bool relu, bf16 *C, int64_t ldc, void *ws, size_t ws_bytes, hipStream_t s) {
    if (!lt || M <= 0 || N <= 0 || K <= 0) return false;
    // one call at a time per handle: the plan's descriptor carries the bias
    std::lock_guard<std::mutex> lock(lt->mu);
    LtPlan *p = nullptr;
    for (auto &q : lt->plans)
        if (q.M == M && q.N == N && q.K == K && q.lda == lda && q.ldw == ldw && q.ldc == ldc &&
            q.bias == (bias != nullptr) && q.relu == relu)
            p = &q;
    const float alpha = 1.f, beta = 0.f;
    auto run = [&](const hipblasLtMatmulAlgo_t &algo, size_t wsz) {
        return hipblasLtMatmul(lt->h, p->desc, &alpha, W, p->la, A, p->lb, &beta, C, p->lc, C, p->lc, &algo, ws, wsz,
                               s) == HIPBLAS_STATUS_SUCCESS;
    };
    if (!p) {
        lt->plans.emplace_back();
        p = &lt->plans.back();
        p->M = M;
        p->N = N;
        p->K = K;
        p->lda = lda;
        p->ldw = ldw;
        p->ldc = ldc;
        p->bias = bias != nullptr;
        p->relu = relu;
        hipblasLtMatmulHeuristicResult_t res[LT_CANDIDATES];
        int got = 0;
        if (!plan(lt, *p, ws_bytes, res, got)) return false;
        if (bias && hipblasLtMatmulDescSetAttribute(p->desc, HIPBLASLT_MATMUL_DESC_BIAS_POINTER, &bias,
                                                    sizeof(bias)) != HIPBLAS_STATUS_SUCCESS)
            return false;
        // the fastest candidate on these operands (a few runs each; the
        // outputs are overwritten by the call's own run), or the heuristic's
        // first while the stream is being captured
        int best = 0;
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (got > 1 && hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone &&
            hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
            float tbest = 0.f;
            for (int i = 0; i < got; ++i) {
                bool ok = run(res[i].algo, res[i].workspaceSize) && hipEventRecord(e0, s) == hipSuccess;
                for (int r = 0; ok && r < 5; ++r) ok = run(res[i].algo, res[i].workspaceSize);
                float ms = 0.f;
                ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (ok && (i == 0 || ms < tbest || tbest == 0.f)) {
                    tbest = ms;
                    best = i;
                }
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        p->algo = res[best].algo;
        p->ws = res[best].workspaceSize;
        p->ok = true;
    }
    if (!p->ok) return false;
    if (bias && hipblasLtMatmulDescSetAttribute(p->desc, HIPBLASLT_MATMUL_DESC_BIAS_POINTER, &bias, sizeof(bias)) !=
                    HIPBLAS_STATUS_SUCCESS)
        return false;
    return run(p->algo, p->ws);
}

}  // namespace pbit
