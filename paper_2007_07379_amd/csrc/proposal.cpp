// Learned proposal object, its training loop and the MH run (host side).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/pbit.h"
#include "blob.h"
#include "made.h"
#include "blaslt.h"
#include "made_kernels.h"
#include "runtime.h"

namespace pbit {
namespace {

// the largest training batch (the gradient's buffers hold this many rows)
constexpr int BATCH_MAX = 16384;
// paths a forward pass of the scorer (and pbit_proposal_logits) takes at
// once: X, H1, H2 and the logits hold this many rows; 65,536 against 16,384
// takes the 131,072-path score of a 1,024-wide network from 1.46 to 1.10 ms
// (four times fewer, larger products and replays)
constexpr int FWD_BATCH = 65536;
static_assert(FWD_BATCH >= BATCH_MAX, "a training batch fits the forward buffers");
// networks up to this width are scored by the fused kernel
constexpr int SCORE_FUSED_MAX_H = 256;

struct DeviceArena {
    std::vector<void *> ptrs;
    ~DeviceArena() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    T *alloc(size_t count) {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return (T *)p;
    }
};

// Scratch of pbit_mh_run_static (the one allocation-free entry point): the
// proposals x', log q(x') and log q(x) of every chain, 4 W + 16 bytes a
// chain.  One array per device, held until the process ends; its device
// address comes from hipGetSymbolAddress (the array's name in host code is
// only a host-side stand-in).  Every call on a device shares it.
constexpr size_t MH_STATIC_BYTES = (size_t)16 << 20;
constexpr int MH_STATIC_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[MH_STATIC_BYTES];
std::mutex g_scratch_mu;
void *g_scratch_ptr[MH_STATIC_DEVICES] = {};

// Device address of `scratch` on device dev, which must be current.
pbit_status static_scratch(int dev, void **out) {
    if (dev < 0 || dev >= MH_STATIC_DEVICES) return set_error(PBIT_E_INVALID_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress of the MH scratch");
        if (!p) return set_error(PBIT_E_DEVICE, "hipGetSymbolAddress returned no address for the MH scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PBIT_OK;
}

int64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return (int64_t)(z ^ (z >> 31));
}

}  // namespace
}  // namespace pbit

using namespace pbit;

struct pbit_proposal_s {
    pbit_circuit circ = nullptr;
    uint32_t idx = 0;
    int D = 0, DP = 0, H = 0, W = 0, h = 0;
    uint64_t P = 0;
    // offsets into the flat parameter vector
    uint64_t oW1, ob1, oW2, ob2, oV, oc;
    std::vector<int> deg_in, deg1, deg2, deg_out, fpos, freem;
    std::vector<int4> phase, phase_k;
    // per free bit, 16 words for the register-resident sampler: the unit
    // ranges {lo1, hi1, lo2, hi2} of its phase, the half tiles of each layer
    // that hold a unit of the phase (bit 2 cc + t) with the layer's K chunk
    // count in the high half, the logit's K chunk count, the lattice
    // position, then the free bit's cone words (W <= 8)
    std::vector<uint32_t> sched;
    // the wide sampler's schedule (SampleArgs::wphase, wstep, wcone)
    std::vector<int4> wphase, wstep;
    std::vector<uint32_t> wcone;
    std::vector<int2> l2;  // its layer-2 steps, {first unit, lo | hi << 8} (the scorer's replay)
    int dev = -1;
    DeviceArena arena;
    // device
    float *theta = nullptr, *m = nullptr, *v = nullptr, *loss = nullptr;
    bf16 *W1b = nullptr, *W1T = nullptr, *W2b = nullptr, *W2T = nullptr, *Vb = nullptr, *VT = nullptr;
    int *d_deg_in = nullptr, *d_deg1 = nullptr, *d_deg2 = nullptr, *d_deg_out = nullptr, *d_free = nullptr,
        *d_fpos = nullptr;
    int *k1end = nullptr, *k2end = nullptr, *k3end = nullptr, *g2beg = nullptr, *g1beg = nullptr;
    int4 *d_phase = nullptr, *d_phase_k = nullptr;
    uint32_t *d_sched = nullptr;
    int4 *d_wphase = nullptr, *d_wstep = nullptr;
    uint32_t *d_wcone = nullptr;
    int2 *d_l2 = nullptr;
    bf16 *X = nullptr, *H1 = nullptr, *H2 = nullptr, *G3 = nullptr, *G2 = nullptr, *G1 = nullptr;
    float *L = nullptr;
    // what the training GEMMs leave for grad_final_kernel: 64-row column
    // partials of G1, G2, G3 (BATCH_MAX / 64 x H, H, D), split-K slices of
    // dW1, dW2, dV (up to zcap[] slices each), the logits tiles' loss shares
    float *cb1 = nullptr, *cb2 = nullptr, *cc = nullptr;
    float *pW1 = nullptr, *pW2 = nullptr, *pV = nullptr;
    int zcap[3] = {0, 0, 0};
    float *losspart = nullptr;
    // the library products of a training step (made on first use; NULL if
    // the library has none for this device) and their workspace
    std::unique_ptr<LtState, void (*)(LtState *)> lt{nullptr, lt_destroy};
    bool lt_tried = false;
    void *lt_ws = nullptr;
    uint32_t *prop = nullptr;
    double *lq_cur = nullptr, *lq_prop = nullptr;
    uint32_t mh_cap = 0;
    int t = 0;  // Adam step
    bool dirty = true;  // bf16 shadows out of date
    std::vector<float> host_params;
};

namespace {

// Weight gradients reduce over the batch (K = n) into few output tiles:
// split K so the launch has about 256 workgroups of 128 x 128 (which the GEMM
// launch then runs as about 1,024 of 64 x 64, four per CU), at most 16
// slices, each of at least four 32-wide chunks.  On the 1,024-wide training
// step, half or twice the slices are 2 % and 5 % slower.
int splitk_slices(int M, int N, int K) {
    const int64_t tiles = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
    const int chunks = (K + 31) / 32;
    const int ks = (int)std::min<int64_t>(16, (256 + tiles - 1) / tiles);
    return std::max(1, std::min(ks, chunks / 4));
}

pbit_status upload(pbit_proposal q, hipStream_t s) {
    if (q->theta) return PBIT_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    q->dev = dev;
    auto &A = q->arena;
    const int D = q->D, DP = q->DP, H = q->H;
    q->theta = A.alloc<float>(q->P);
    q->m = A.alloc<float>(q->P);
    q->v = A.alloc<float>(q->P);
    q->loss = A.alloc<float>(1 << 16);
    q->W1b = A.alloc<bf16>((size_t)D * H);
    q->W1T = A.alloc<bf16>((size_t)H * DP);
    q->W2b = A.alloc<bf16>((size_t)H * H);
    q->W2T = A.alloc<bf16>((size_t)H * H);
    q->Vb = A.alloc<bf16>((size_t)H * D);
    q->VT = A.alloc<bf16>((size_t)D * H);
    q->X = A.alloc<bf16>((size_t)FWD_BATCH * DP);
    q->H1 = A.alloc<bf16>((size_t)FWD_BATCH * H);
    q->H2 = A.alloc<bf16>((size_t)FWD_BATCH * H);
    q->G1 = A.alloc<bf16>((size_t)BATCH_MAX * H);
    q->G2 = A.alloc<bf16>((size_t)BATCH_MAX * H);
    q->G3 = A.alloc<bf16>((size_t)BATCH_MAX * D);
    q->L = A.alloc<float>((size_t)FWD_BATCH * D);
    q->cb1 = A.alloc<float>((size_t)(BATCH_MAX / 64) * H);
    q->cb2 = A.alloc<float>((size_t)(BATCH_MAX / 64) * H);
    q->cc = A.alloc<float>((size_t)(BATCH_MAX / 64) * D);
    // slices for the largest batch (the split only grows with K)
    q->zcap[0] = splitk_slices(D, H, BATCH_MAX);
    q->zcap[1] = splitk_slices(H, H, BATCH_MAX);
    q->zcap[2] = splitk_slices(H, D, BATCH_MAX);
    q->pW1 = A.alloc<float>((size_t)q->zcap[0] * D * H);
    q->pW2 = A.alloc<float>((size_t)q->zcap[1] * H * H);
    q->pV = A.alloc<float>((size_t)q->zcap[2] * H * D);
    q->losspart = A.alloc<float>((size_t)(BATCH_MAX / 64) * ((D + 63) / 64));
    q->lt_ws = A.alloc<unsigned char>(LT_WORKSPACE);
    hipError_t ce = hipSuccess;  // first failure of the copies below
    auto copy = [&](void *dst, const void *src, size_t bytes) {
        if (ce == hipSuccess && dst && bytes) ce = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    auto up = [&](int *&dst, const std::vector<int> &src) {
        dst = A.alloc<int>(src.size() + 64);
        copy(dst, src.data(), src.size() * sizeof(int));
    };
    up(q->d_deg_in, q->deg_in);
    up(q->d_deg1, q->deg1);
    up(q->d_deg2, q->deg2);
    up(q->d_deg_out, q->deg_out);
    up(q->d_free, q->freem);
    up(q->d_fpos, q->fpos);
    // per 64-column tile reduction ranges (masked weights are zero outside)
    auto count_le = [](const std::vector<int> &deg, int v) {
        return (int)(std::upper_bound(deg.begin(), deg.end(), v) - deg.begin());
    };
    std::vector<int> k1, k2, k3, b2, b1;
    for (int nt = 0; nt * 64 < H; ++nt) {
        const int last = std::min(nt * 64 + 63, H - 1);
        k1.push_back(q->deg1[last]);
        k2.push_back(count_le(q->deg1, q->deg2[last]));
        b2.push_back(q->deg2[nt * 64]);  // G2 column u2 sums over o >= deg2(u2)
        b1.push_back((int)(std::lower_bound(q->deg2.begin(), q->deg2.end(), q->deg1[nt * 64]) - q->deg2.begin()));
    }
    for (int nt = 0; nt * 64 < D; ++nt) {
        const int last = std::min(nt * 64 + 63, D - 1);
        k3.push_back(count_le(q->deg2, last));
    }
    up(q->k1end, k1);
    up(q->k2end, k2);
    up(q->k3end, k3);
    up(q->g2beg, b2);
    up(q->g1beg, b1);
    q->d_phase = A.alloc<int4>(q->phase.size() + 1);
    q->d_phase_k = A.alloc<int4>(q->phase_k.size() + 1);
    q->d_sched = A.alloc<uint32_t>(q->sched.size() + 16);
    q->d_wphase = A.alloc<int4>(q->wphase.size() + 1);
    q->d_wstep = A.alloc<int4>(q->wstep.size() + 1);
    q->d_wcone = A.alloc<uint32_t>(q->wcone.size() + 1);
    q->d_l2 = A.alloc<int2>(q->l2.size() + 1);
    if (!q->theta || !q->L || !q->cb1 || !q->cb2 || !q->cc || !q->pW1 || !q->pW2 || !q->pV || !q->losspart ||
        !q->lt_ws || !q->m || !q->v || !q->loss || !q->W1b || !q->W1T || !q->W2b || !q->W2T || !q->Vb || !q->VT ||
        !q->X || !q->H1 || !q->H2 || !q->G1 || !q->G2 || !q->G3 ||
        !q->d_phase || !q->d_phase_k || !q->g1beg ||
        !q->d_sched || !q->d_wphase || !q->d_wstep || !q->d_wcone || !q->d_l2)
        return set_error(PBIT_E_OOM, "device allocation for the proposal failed");
    copy(q->d_sched, q->sched.data(), q->sched.size() * sizeof(uint32_t));
    copy(q->d_wphase, q->wphase.data(), q->wphase.size() * sizeof(int4));
    copy(q->d_wstep, q->wstep.data(), q->wstep.size() * sizeof(int4));
    copy(q->d_wcone, q->wcone.data(), q->wcone.size() * sizeof(uint32_t));
    copy(q->d_l2, q->l2.data(), q->l2.size() * sizeof(int2));
    copy(q->d_phase, q->phase.data(), q->phase.size() * sizeof(int4));
    copy(q->d_phase_k, q->phase_k.data(), q->phase_k.size() * sizeof(int4));
    copy(q->theta, q->host_params.data(), q->P * sizeof(float));
    if (ce != hipSuccess) return hip_error(ce, "proposal upload");
    // Adam moments start at zero
    e = hipMemsetAsync(q->m, 0, q->P * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(q->v, 0, q->P * sizeof(float), s);
    // later calls may come on other streams: the set-up is complete on return
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "proposal upload");
    return PBIT_OK;
}

pbit_status refresh(pbit_proposal q, hipStream_t s) {
    if (!q->dirty) return PBIT_OK;
    q->dirty = false;
    hipError_t e;
    ShadowJobs jobs;
    jobs.j[0] = {q->theta + q->oW1, q->D, q->H, q->DP, q->W1b, q->W1T};
    jobs.j[1] = {q->theta + q->oW2, q->H, q->H, q->H, q->W2b, q->W2T};
    jobs.j[2] = {q->theta + q->oV, q->H, q->D, q->H, q->Vb, q->VT};
    if ((e = launch_shadow(jobs, 3, s)) != hipSuccess) return hip_error(e, "shadow refresh");
    return PBIT_OK;
}

GemmArgs gemm0() {
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    return g;
}

// A weight gradient's GEMM leaves its split-K slices in `part` (up to cap
// of them); returns the slice count.
int splitk(GemmArgs &g, float *part, int cap) {
    const int ks = std::min(splitk_slices(g.M, g.N, g.K), cap);
    g.ksplit = ks;
    g.keep_parts = 1;
    g.part = part;
    return ks;
}

// Forward of n <= FWD_BATCH paths (X already unpacked): H1, H2, L (a
// training step: n <= BATCH_MAX).
// The library handle of a training step's products (NULL when there is none).
LtState *lt_of(pbit_proposal q) {
    if (!q->lt_tried) {
        q->lt_tried = true;
        q->lt.reset(lt_create());
    }
    return q->lt.get();
}

// The network on the batch in q->X.  For the wide sampler's scorer (wide):
// layer 2 in the sampler's k-slot order, and no logits (the replay adds
// them in the sampler's order).  For training (train): the logits GEMM
// writes the loss gradient G3 (bf16), its column partials and the loss
// shares instead of the logits.
pbit_status forward(pbit_proposal q, int n, hipStream_t s, bool wide = false, bool train = false) {
    const int D = q->D, DP = q->DP, H = q->H;
    // a training step's hidden layers: the library products when they run
    LtState *lt = train ? lt_of(q) : nullptr;
    const bool lt_hidden =
        lt &&
        lt_gemm_nt(lt, n, H, DP, q->X, DP, q->W1T, DP, q->theta + q->ob1, true, q->H1, H, q->lt_ws, LT_WORKSPACE, s) &&
        lt_gemm_nt(lt, n, H, H, q->H1, H, q->W2T, H, q->theta + q->ob2, true, q->H2, H, q->lt_ws, LT_WORKSPACE, s);
    GemmArgs g;
    hipError_t e;
    if (!lt_hidden) {
        g = gemm0();
        g.A = q->X; g.sam = DP; g.sak = 1;
        g.B = q->W1T; g.sbk = 1; g.sbn = DP;
        g.C = q->H1; g.scm = H; g.scn = 1;
        g.M = n; g.N = H; g.K = D;
        g.kend = q->k1end; g.bias = q->theta + q->ob1; g.relu = 1; g.out_bf16 = 1;
        if ((e = launch_gemm(g, s)) != hipSuccess) return hip_error(e, "gemm1");
        g = gemm0();
        g.A = q->H1; g.sam = H; g.sak = 1;
        g.B = q->W2T; g.sbk = 1; g.sbn = H;
        g.C = q->H2; g.scm = H; g.scn = 1;
        g.M = n; g.N = H; g.K = H;
        g.kend = q->k2end; g.bias = q->theta + q->ob2; g.relu = 1; g.out_bf16 = 1;
        g.kperm = wide ? 1 : 0;
        if ((e = launch_gemm(g, s)) != hipSuccess) return hip_error(e, "gemm2");
    }
    if (wide) return PBIT_OK;
    g = gemm0();
    g.A = q->H2; g.sam = H; g.sak = 1;
    g.B = q->VT; g.sbk = 1; g.sbn = H;
    g.C = q->L; g.scm = D; g.scn = 1;
    g.M = n; g.N = D; g.K = H;
    g.kend = q->k3end; g.bias = q->theta + q->oc; g.out_bf16 = 0;
    if (train) {
        g.C = q->G3;
        g.out_bf16 = 1;
        g.lossx = q->X;
        g.slx = DP;
        g.lossfree = q->d_free;
        g.inv_n = 1.f / (float)n;
        g.losspart = q->losspart;
        g.colpart = q->cc;
    }
    if ((e = launch_gemm(g, s)) != hipSuccess) return hip_error(e, "gemm3");
    return PBIT_OK;
}

// The backward GEMMs of the batch after forward(train): the weight
// gradients' split-K slices into pW1, pW2, pV (slice counts into z[]) and
// the column partials of G2, G1 into cb2, cb1; grad_final finishes them.
pbit_status backward(pbit_proposal q, int n, hipStream_t s, int z[3]) {
    const int D = q->D, DP = q->DP, H = q->H;
    hipError_t e;
    GemmArgs g;
    // G2 = (G3 V^T) * (H2 > 0); db2 partials (the library product, then the
    // gate and the column partials, when it runs)
    LtState *lt = lt_of(q);
    if (lt && lt_gemm_nt(lt, n, H, D, q->G3, D, q->Vb, D, nullptr, false, q->G2, H, q->lt_ws, LT_WORKSPACE, s)) {
        if ((e = launch_gate_colsum(q->G2, q->H2, n, H, q->cb2, s)) != hipSuccess) return hip_error(e, "G2 gate");
    } else {
        g = gemm0();
        g.A = q->G3; g.sam = D; g.sak = 1;
        g.B = q->Vb; g.sbk = 1; g.sbn = D;
        g.C = q->G2; g.scm = H; g.scn = 1;
        g.M = n; g.N = H; g.K = D;
        g.kbeg = q->g2beg; g.gate = q->H2; g.sgm = H; g.sgn = 1; g.out_bf16 = 1;
        g.colpart = q->cb2;
        if ((e = launch_gemm(g, s)) != hipSuccess) return hip_error(e, "G2");
    }
    // G1 = (G2 W2^T) * (H1 > 0); db1 partials
    if (lt && lt_gemm_nt(lt, n, H, H, q->G2, H, q->W2b, H, nullptr, false, q->G1, H, q->lt_ws, LT_WORKSPACE, s)) {
        if ((e = launch_gate_colsum(q->G1, q->H1, n, H, q->cb1, s)) != hipSuccess) return hip_error(e, "G1 gate");
    } else {
        g = gemm0();
        g.A = q->G2; g.sam = H; g.sak = 1;
        g.B = q->W2b; g.sbk = 1; g.sbn = H;
        g.C = q->G1; g.scm = H; g.scn = 1;
        g.M = n; g.N = H; g.K = H;
        g.kbeg = q->g1beg; g.gate = q->H1; g.sgm = H; g.sgn = 1; g.out_bf16 = 1;
        g.colpart = q->cb1;
        if ((e = launch_gemm(g, s)) != hipSuccess) return hip_error(e, "G1");
    }
    // the weight gradients, split-K slices kept for grad_final: dW2 = H1^T G2,
    // dV = H2^T G3, dW1 = X^T G1 (masked), in one launch (dW2, whose slices
    // are the longest, first)
    GemmArgs w[3];
    w[0] = gemm0();
    w[0].A = q->H1; w[0].sam = 1; w[0].sak = H;
    w[0].B = q->G2; w[0].sbk = H; w[0].sbn = 1;
    w[0].M = H; w[0].N = H; w[0].K = n;
    w[0].deg_row = q->d_deg1; w[0].deg_col = q->d_deg2;
    z[1] = splitk(w[0], q->pW2, q->zcap[1]);
    w[1] = gemm0();
    w[1].A = q->H2; w[1].sam = 1; w[1].sak = H;
    w[1].B = q->G3; w[1].sbk = D; w[1].sbn = 1;
    w[1].M = H; w[1].N = D; w[1].K = n;
    w[1].deg_row = q->d_deg2; w[1].deg_col = q->d_deg_out;
    z[2] = splitk(w[1], q->pV, q->zcap[2]);
    w[2] = gemm0();
    w[2].A = q->X; w[2].sam = 1; w[2].sak = DP;
    w[2].B = q->G1; w[2].sbk = H; w[2].sbn = 1;
    w[2].M = D; w[2].N = H; w[2].K = n;
    w[2].deg_row = q->d_deg_in; w[2].deg_col = q->d_deg1;
    z[0] = splitk(w[2], q->pW1, q->zcap[0]);
    if ((e = launch_gemm_group(w, 3, s)) != hipSuccess) return hip_error(e, "weight gradients");
    return PBIT_OK;
}

// The gradient of the batch of n into `grad` (adam_step == false), or one
// Adam step on it that also writes the weights' bf16 shadows; the batch-mean
// loss into *loss_dev.
pbit_status grad_final(pbit_proposal q, int n, const int z[3], float *loss_dev, bool adam_step, float *grad, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s,
                       const uint32_t *next_states = nullptr, uint64_t next_stride = 0, uint64_t next_b0 = 0,
                       int next_n = 0) {
    GradFinal a;
    std::memset(&a, 0, sizeof(a));
    a.adam = adam_step ? 1 : 0;
    a.th = q->theta;
    a.m = q->m;
    a.v = q->v;
    a.grad = grad;
    a.lr = lr;
    a.b1 = b1;
    a.b2 = b2;
    a.eps = eps;
    a.c1 = c1;
    a.c2 = c2;
    a.P = (int64_t)q->P;
    a.oW1 = (int64_t)q->oW1;
    a.ob1 = (int64_t)q->ob1;
    a.oW2 = (int64_t)q->oW2;
    a.ob2 = (int64_t)q->ob2;
    a.oV = (int64_t)q->oV;
    a.oc = (int64_t)q->oc;
    a.D = q->D;
    a.H = q->H;
    a.pW1 = q->pW1;
    a.pW2 = q->pW2;
    a.pV = q->pV;
    a.zW1 = z[0];
    a.zW2 = z[1];
    a.zV = z[2];
    a.cb1 = q->cb1;
    a.cb2 = q->cb2;
    a.cc = q->cc;
    a.chunks = (n + 63) / 64;
    a.deg_in = q->d_deg_in;
    a.deg1 = q->d_deg1;
    a.deg2 = q->d_deg2;
    a.deg_out = q->d_deg_out;
    a.losspart = q->losspart;
    a.nloss = ((n + 63) / 64) * ((q->D + 63) / 64);
    a.loss = loss_dev;
    if (adam_step) {  // the step writes the shadows of the updated weights
        a.sh[0] = {nullptr, q->D, q->H, q->DP, q->W1b, q->W1T};
        a.sh[1] = {nullptr, q->H, q->H, q->H, q->W2b, q->W2T};
        a.sh[2] = {nullptr, q->H, q->D, q->H, q->Vb, q->VT};
        if (next_n > 0) {  // the next batch's inputs, unpacked in the same launch
            a.ux_states = next_states;
            a.ux_stride = next_stride;
            a.ux_b0 = next_b0;
            a.ux_n = next_n;
            a.ux_DP = q->DP;
            a.ux_X = q->X;
        }
    }
    hipError_t e = launch_grad_final(a, s);
    if (e != hipSuccess) return hip_error(e, adam_step ? "adam" : "gradient");
    return PBIT_OK;
}

pbit_status unpack_range(pbit_proposal q, const uint32_t *states, uint64_t stride, uint64_t b0, int n,
                         hipStream_t s);
pbit_status sample_or_score(pbit_proposal q, uint32_t n, uint32_t chain_begin, uint64_t seed, uint32_t step,
                            uint32_t *d_out, double *d_logq, const uint32_t *score, hipStream_t hip_stream,
                            double *d_logq_cur = nullptr);

}  // namespace

// unpack of a column range of a word-major state array with row stride
// `stride` (unpack_row8 per thread).  DP is a multiple of 32 and n DP / 8 <
// 2^32 (checked at launch).
__global__ void unpack_strided_kernel(const uint32_t *__restrict__ states, uint64_t stride, uint64_t b0, int n,
                                      int D, int DP, bf16 *__restrict__ X) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint32_t)n * ((uint32_t)DP >> 3)) return;
    unpack_row8(states, stride, b0, D, DP, X, e);
}

__global__ void fill_const_kernel(const uint32_t *__restrict__ blob, uint32_t *__restrict__ state, int n, int W) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * W) return;
    const int w = (int)(e / n);
    state[e] = blob[blob[H_OFF_CONST] + w];
}

namespace {
pbit_status unpack_range(pbit_proposal q, const uint32_t *states, uint64_t stride, uint64_t b0, int n,
                         hipStream_t s) {
    const int64_t tot = (int64_t)n * (q->DP / 8);
    if (q->DP % 32 || tot > (int64_t)UINT32_MAX) return set_error(PBIT_E_INVALID_ARG, "unpack: bad row length or batch");
    if (tot == 0) return PBIT_OK;
    hipLaunchKernelGGL(unpack_strided_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, states, stride, b0,
                       n, q->D, q->DP, q->X);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "unpack");
    return PBIT_OK;
}
}  // namespace

extern "C" {

pbit_status pbit_proposal_create(pbit_circuit c, uint32_t idx, const pbit_made_cfg *cfg, pbit_proposal *out) {
    if (!out) return set_error(PBIT_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!c || idx >= c->circuits.size()) return set_error(PBIT_E_INVALID_ARG, "bad circuit handle or index");
    const CompiledCircuit &k = c->circuits[idx];
    const uint32_t H = cfg && cfg->hidden ? cfg->hidden : 1024;
    if (H % 64 || H > 4096) return set_error(PBIT_E_INVALID_ARG, "hidden must be a multiple of 64, <= 4096");
    if (k.h == 0) return set_error(PBIT_E_INVALID_ARG, "circuit has no free p-bit");
    if (k.ny)
        return set_error(PBIT_E_MODE_UNAVAILABLE,
                         "the proposal builds paths through cones; three-qubit products are not affine");
    if (k.blob[H_NSOFT])
        return set_error(PBIT_E_MODE_UNAVAILABLE, "soft zeros: the MH chain would bin paths that meet them");
    {
        SampleArgs probe;
        std::memset(&probe, 0, sizeof(probe));
        probe.n = 1;
        probe.h = (int)k.h;
        probe.W = (int)k.W;
        probe.D = (int)k.L;
        probe.DP = ((int)k.L + 31) / 32 * 32;
        probe.H = (int)H;
        if (!made_sample_launchable(probe))
            return set_error(PBIT_E_TOO_LARGE, "hidden width " + std::to_string(H) + " over " + std::to_string(k.L) +
                                                   " lattice positions: the sampler's activations exceed 160 KiB of LDS");
    }
    auto *q = new pbit_proposal_s();
    q->circ = c;
    q->idx = idx;
    q->D = (int)k.L;
    q->DP = (q->D + 31) / 32 * 32;
    q->H = (int)H;
    q->W = (int)k.W;
    q->h = (int)k.h;
    const int D = q->D;
    q->oW1 = 0;
    q->ob1 = q->oW1 + (uint64_t)D * H;
    q->oW2 = q->ob1 + H;
    q->ob2 = q->oW2 + (uint64_t)H * H;
    q->oV = q->ob2 + H;
    q->oc = q->oV + (uint64_t)H * D;
    q->P = q->oc + D;
    for (int i = 0; i < D; ++i) q->deg_in.push_back(i + 1);
    for (uint32_t u = 0; u < H; ++u) q->deg1.push_back(1 + (int)(((uint64_t)u * (uint64_t)(D - 1)) / H));
    q->deg2 = q->deg1;
    for (int o = 0; o < D; ++o) q->deg_out.push_back(o);
    q->freem.assign(D, 0);
    const uint32_t *fp = k.blob.data() + k.blob[H_OFF_FPOS];
    for (uint32_t b = 0; b < k.h; ++b) {
        q->fpos.push_back((int)fp[b]);
        q->freem[fp[b]] = 1;
    }
    // sampler phases: units whose degree falls in (previous free position, p]
    auto count_le = [](const std::vector<int> &deg, int v) {
        return (int)(std::upper_bound(deg.begin(), deg.end(), v) - deg.begin());
    };
    int prev = 0;
    for (uint32_t b = 0; b < k.h; ++b) {
        const int p = q->fpos[b];
        const int u1a = count_le(q->deg1, prev), u1b = count_le(q->deg1, p);
        const int u2a = count_le(q->deg2, prev), u2b = count_le(q->deg2, p);
        const int k1 = u1b > u1a ? q->deg1[u1b - 1] : 0;
        const int k2 = u2b > u2a ? count_le(q->deg1, q->deg2[u2b - 1]) : 0;
        const int k3 = count_le(q->deg2, p);
        q->phase.push_back(int4{u1a, u1b, u2a, u2b});
        q->phase_k.push_back(int4{k1, k2, k3, p});
        prev = p;
        uint32_t m1 = 0, m2 = 0;  // half tile 2 cc + t holds the 16 units 32 cc + 16 t ..
        for (int u = u1a; u < u1b; ++u) m1 |= 1u << (u >> 4);
        for (int u = u2a; u < u2b; ++u) m2 |= 1u << (u >> 4);
        const uint32_t rec[8] = {(uint32_t)u1a, (uint32_t)u1b, (uint32_t)u2a, (uint32_t)u2b,
                                 (m1 & 0xffffu) | ((uint32_t)((k1 + 31) / 32) << 16),
                                 (m2 & 0xffffu) | ((uint32_t)((k2 + 31) / 32) << 16), (uint32_t)((k3 + 31) / 32),
                                 (uint32_t)p};
        for (uint32_t r : rec) q->sched.push_back(r);
        // the wide sampler's steps: the layer-1 half tiles holding a unit of
        // the phase, then the layer-2 ones with the phase's units among their
        // 16 ([lo, hi) as lo | hi << 8), whose logit terms are added then
        const int s0 = (int)q->wstep.size();
        // (K chunks rounded up to a multiple of 8 within the row: the extra
        // chunks meet weights the degree masks keep at zero)
        const int nk1 = std::min((k1 + 255) / 256 * 8, q->DP / 32), nk2 = std::min((k2 + 255) / 256 * 8, (int)H / 32);
        if (u1b > u1a)
            for (int ht = u1a / 16; ht <= (u1b - 1) / 16; ++ht) q->wstep.push_back(int4{0, 16 * ht, nk1, 0});
        if (u2b > u2a)
            for (int ht = u2a / 16; ht <= (u2b - 1) / 16; ++ht) {
                const int lo = std::max(u2a - 16 * ht, 0), hi = std::min(u2b - 16 * ht, 16);
                q->wstep.push_back(int4{1, 16 * ht, nk2, lo | hi << 8});
                q->l2.push_back(int2{16 * ht, lo | hi << 8});
            }
        q->wphase.push_back(int4{s0, (int)q->wstep.size(), p, 0});
        const uint32_t *cn = k.blob.data() + k.blob[H_OFF_CONE] + (size_t)b * k.WS;
        for (uint32_t w = 0; w < 8; ++w) q->sched.push_back(w < k.W ? cn[w] : 0u);
        // at least 16 words a free bit, zero past W, so the wide sampler
        // reads a fixed-length block
        for (uint32_t w = 0; w < wd_cone_stride(k.W); ++w) q->wcone.push_back(w < k.W ? cn[w] : 0u);
    }
    // initial parameters
    q->host_params.assign(q->P, 0.f);
    uint64_t st = cfg ? cfg->seed : 0;
    auto init = [&](uint64_t off, int K, int N, const std::vector<int> &dr, const std::vector<int> &dc) {
        const float a = 1.0f / std::sqrt((float)K);
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < N; ++j) {
                const double u = (double)((uint64_t)splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
                q->host_params[off + (uint64_t)i * N + j] = dr[i] <= dc[j] ? (float)((2.0 * u - 1.0) * a) : 0.f;
            }
    };
    init(q->oW1, D, (int)H, q->deg_in, q->deg1);
    init(q->oW2, (int)H, (int)H, q->deg1, q->deg2);
    init(q->oV, (int)H, D, q->deg2, q->deg_out);
    // set-up on the current device: the network and its work buffers, the
    // circuit images, and the address of the allocation-free MH scratch
    pbit_status ps = upload(q, nullptr);
    const uint32_t *dblob = nullptr;
    if (ps == PBIT_OK) {
        std::lock_guard<std::mutex> lock(c->mu);
        ps = device_blobs(c, &dblob);
    }
    void *scr = nullptr;
    if (ps == PBIT_OK) ps = static_scratch(q->dev, &scr);
    if (ps != PBIT_OK) {
        delete q;
        return ps;
    }
    *out = q;
    return PBIT_OK;
}

void pbit_proposal_free(pbit_proposal q) { delete q; }

pbit_status pbit_proposal_info(pbit_proposal q, uint32_t *D, uint32_t *H, uint64_t *n_params) {
    if (!q) return set_error(PBIT_E_INVALID_ARG, "NULL proposal");
    if (D) *D = (uint32_t)q->D;
    if (H) *H = (uint32_t)q->H;
    if (n_params) *n_params = q->P;
    return PBIT_OK;
}

pbit_status pbit_proposal_set_params(pbit_proposal q, const float *params, uint64_t n) {
    if (!q || !params || n != q->P) return set_error(PBIT_E_INVALID_ARG, "bad proposal or parameter count");
    q->host_params.assign(params, params + n);
    // keep masked weights at exactly zero
    auto mask = [&](uint64_t off, int K, int N, const std::vector<int> &dr, const std::vector<int> &dc) {
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < N; ++j)
                if (dr[i] > dc[j]) q->host_params[off + (uint64_t)i * N + j] = 0.f;
    };
    mask(q->oW1, q->D, q->H, q->deg_in, q->deg1);
    mask(q->oW2, q->H, q->H, q->deg1, q->deg2);
    mask(q->oV, q->H, q->D, q->deg2, q->deg_out);
    q->t = 0;
    q->dirty = true;
    if (q->theta) {
        hipError_t e = hipMemcpy(q->theta, q->host_params.data(), q->P * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(q->m, 0, q->P * sizeof(float));
        if (e == hipSuccess) e = hipMemset(q->v, 0, q->P * sizeof(float));
        if (e != hipSuccess) return hip_error(e, "set_params");
    }
    return PBIT_OK;
}

pbit_status pbit_proposal_get_params(pbit_proposal q, float *params, uint64_t n) {
    if (!q || !params || n != q->P) return set_error(PBIT_E_INVALID_ARG, "bad proposal or parameter count");
    if (q->theta) {
        hipError_t e = hipMemcpy(params, q->theta, q->P * sizeof(float), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_error(e, "get_params");
    } else {
        std::memcpy(params, q->host_params.data(), q->P * sizeof(float));
    }
    return PBIT_OK;
}

pbit_status pbit_proposal_logits(pbit_proposal q, const uint32_t *d_states, uint32_t n, float *d_logits,
                                 void *hip_stream) {
    if (!q || !d_states || !d_logits) return set_error(PBIT_E_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)hip_stream;
    pbit_status st = upload(q, s);
    if (st != PBIT_OK) return st;
    if ((st = refresh(q, s)) != PBIT_OK) return st;
    for (uint32_t b0 = 0; b0 < n; b0 += FWD_BATCH) {
        const int nb = (int)std::min<uint32_t>(FWD_BATCH, n - b0);
        if ((st = unpack_range(q, d_states, n, b0, nb, s)) != PBIT_OK) return st;
        if ((st = forward(q, nb, s)) != PBIT_OK) return st;
        hipError_t e = hipMemcpyAsync(d_logits + (uint64_t)b0 * q->D, q->L, (size_t)nb * q->D * sizeof(float),
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_error(e, "logits copy");
    }
    return PBIT_OK;
}

pbit_status pbit_proposal_grad(pbit_proposal q, const uint32_t *d_states, uint32_t n, float *d_grad,
                               float *loss_out, void *hip_stream) {
    if (!q || !d_states || !d_grad) return set_error(PBIT_E_INVALID_ARG, "NULL argument");
    if (n == 0 || n > (uint32_t)BATCH_MAX) return set_error(PBIT_E_INVALID_ARG, "batch must be 1..16384");
    hipStream_t s = (hipStream_t)hip_stream;
    pbit_status st = upload(q, s);
    if (st != PBIT_OK) return st;
    if ((st = refresh(q, s)) != PBIT_OK) return st;
    if ((st = unpack_range(q, d_states, n, 0, (int)n, s)) != PBIT_OK) return st;
    if ((st = forward(q, (int)n, s, false, true)) != PBIT_OK) return st;
    int z[3];
    if ((st = backward(q, (int)n, s, z)) != PBIT_OK) return st;
    if ((st = grad_final(q, (int)n, z, q->loss, false, d_grad, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, s)) != PBIT_OK) return st;
    float l = 0.f;
    hipError_t e;
    e = hipMemcpyAsync(&l, q->loss, sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_error(e, "loss copy");
    if (loss_out) *loss_out = l;
    return PBIT_OK;
}

pbit_status pbit_proposal_train(pbit_proposal q, const uint32_t *d_states, uint64_t n_samples,
                                const pbit_train_cfg *cfg, float *losses_out, void *hip_stream) {
    if (!q || !d_states || !cfg) return set_error(PBIT_E_INVALID_ARG, "NULL argument");
    if (cfg->batch == 0 || cfg->batch > (uint32_t)BATCH_MAX || cfg->batch > n_samples)
        return set_error(PBIT_E_INVALID_ARG, "batch must be 1..min(16384, n_samples)");
    if (cfg->steps > (1u << 16)) return set_error(PBIT_E_INVALID_ARG, "at most 65536 steps per call");
    const float lr = cfg->lr > 0 ? cfg->lr : 1e-3f, b1 = cfg->beta1 > 0 ? cfg->beta1 : 0.9f;
    const float b2 = cfg->beta2 > 0 ? cfg->beta2 : 0.999f, eps = cfg->eps > 0 ? cfg->eps : 1e-8f;
    hipStream_t s = (hipStream_t)hip_stream;
    pbit_status st = upload(q, s);
    if (st != PBIT_OK) return st;
    if ((st = refresh(q, s)) != PBIT_OK) return st;
    hipError_t e = hipMemsetAsync(q->loss, 0, sizeof(float) * cfg->steps, s);
    if (e != hipSuccess) return hip_error(e, "memset");
    // consecutive batches, wrapping to the start when one would run past the
    // samples; each step's finalize unpacks the next step's batch (X is last
    // read by that step's weight gradients), the first is unpacked here
    auto wrap = [&](uint64_t c) { return c + cfg->batch > n_samples ? (uint64_t)0 : c; };
    uint64_t cursor = wrap(0);
    if (cfg->steps && (st = unpack_range(q, d_states, n_samples, cursor, (int)cfg->batch, s)) != PBIT_OK) return st;
    for (uint32_t it = 0; it < cfg->steps; ++it) {
        if ((st = forward(q, (int)cfg->batch, s, false, true)) != PBIT_OK) return st;
        int z[3];
        if ((st = backward(q, (int)cfg->batch, s, z)) != PBIT_OK) return st;
        q->t += 1;
        const double c1 = 1.0 / (1.0 - std::pow((double)b1, q->t));
        const double c2 = 1.0 / (1.0 - std::pow((double)b2, q->t));
        const uint64_t next = wrap(cursor + cfg->batch);
        const bool more = it + 1 < cfg->steps;
        if ((st = grad_final(q, (int)cfg->batch, z, q->loss + it, true, nullptr, lr, b1, b2, eps, (float)c1,
                             (float)c2, s, more ? d_states : nullptr, n_samples, next, more ? (int)cfg->batch : 0)) !=
            PBIT_OK)
            return st;
        cursor = next;
        q->dirty = false;  // the Adam step refreshed the shadows
    }
    if (losses_out) {
        e = hipMemcpyAsync(losses_out, q->loss, sizeof(float) * cfg->steps, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_error(e, "loss copy");
    }
    return PBIT_OK;
}

pbit_status pbit_proposal_sample(pbit_proposal q, uint32_t n, uint32_t chain_begin, uint64_t seed, uint32_t step,
                                 uint32_t *d_out, double *d_logq, void *hip_stream) {
    if (!q || !d_out || !d_logq) return set_error(PBIT_E_INVALID_ARG, "NULL argument");
    return sample_or_score(q, n, chain_begin, seed, step, d_out, d_logq, nullptr, (hipStream_t)hip_stream);
}

}  // extern "C"

namespace {

// The fused autoregressive kernel: draws paths (score == NULL) or reads
// their bits from `score` and returns log q with the same arithmetic.
pbit_status sample_or_score(pbit_proposal q, uint32_t n, uint32_t chain_begin, uint64_t seed, uint32_t step,
                            uint32_t *d_out, double *d_logq, const uint32_t *score, hipStream_t hip_stream,
                            double *d_logq_cur) {
    if ((uint64_t)chain_begin + n > 0x100000000ull) return set_error(PBIT_E_INVALID_ARG, "chain index overflow");
    hipStream_t s = (hipStream_t)hip_stream;
    pbit_status st = upload(q, s);
    if (st != PBIT_OK) return st;
    if ((st = refresh(q, s)) != PBIT_OK) return st;
    const uint32_t *dblob = nullptr;
    {
        std::lock_guard<std::mutex> lock(q->circ->mu);
        if ((st = device_blobs(q->circ, &dblob)) != PBIT_OK) return st;
    }
    SampleArgs a;
    std::memset(&a, 0, sizeof(a));
    a.blob = dblob + q->circ->blob_off[q->idx];
    a.W1T = q->W1T;
    a.W2T = q->W2T;
    a.VT = q->VT;
    a.b1 = q->theta + q->ob1;
    a.b2 = q->theta + q->ob2;
    a.c = q->theta + q->oc;
    a.phase = q->d_phase;
    a.phase_k = q->d_phase_k;
    a.sched = q->d_sched;
    a.n = (int)n;
    a.h = q->h;
    a.W = q->W;
    a.D = q->D;
    a.DP = q->DP;
    a.H = q->H;
    a.chain_begin = chain_begin;
    a.step = step;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.out = d_out;
    a.logq = d_logq;
    a.score = score;
    a.logq_cur = d_logq_cur;
    a.wphase = q->d_wphase;
    a.wstep = q->d_wstep;
    a.wcone = q->d_wcone;
    a.cone_stride = wd_cone_stride(q->W);
    a.nsteps = (int)q->wstep.size();
    if (d_logq_cur) {
        hipError_t e = launch_made_sample_dual(a, s);
        if (e != hipSuccess) return hip_error(e, "made sampler (sample and score)");
        return PBIT_OK;
    }
    hipError_t e = launch_made_sample(a, s);
    if (e != hipSuccess) return hip_error(e, "made sampler");
    return PBIT_OK;
}

}  // namespace

extern "C" {

pbit_status pbit_proposal_score(pbit_proposal q, const uint32_t *d_states, uint32_t n, double *d_logq,
                                void *hip_stream) {
    if (!q || !d_states || !d_logq) return set_error(PBIT_E_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)hip_stream;
    // small networks: the sampler's own kernel in score mode.  Else the
    // batched GEMMs, whose activations carry the samplers' bits, then the
    // logits in the order of the sampler that serves the shape: the wide
    // sampler's replay, or one more GEMM (made_sample_kernel's order).  The
    // scorer gives the sampler's bits either way.
    if (q->H <= SCORE_FUSED_MAX_H) return sample_or_score(q, n, 0, 0, 0, nullptr, d_logq, d_states, s);
    SampleArgs probe;
    std::memset(&probe, 0, sizeof(probe));
    probe.H = q->H;
    probe.h = q->h;
    probe.W = q->W;
    probe.D = q->D;
    probe.DP = q->DP;
    const bool wide = made_sample_wide_ok(probe);
    pbit_status st = upload(q, s);
    if (st != PBIT_OK) return st;
    if ((st = refresh(q, s)) != PBIT_OK) return st;
    for (uint32_t b0 = 0; b0 < n; b0 += FWD_BATCH) {
        const int nb = (int)std::min<uint32_t>(FWD_BATCH, n - b0);
        if ((st = unpack_range(q, d_states, n, b0, nb, s)) != PBIT_OK) return st;
        if ((st = forward(q, nb, s, wide)) != PBIT_OK) return st;
        hipError_t e;
        if (wide) {
            ReplayArgs r;
            r.H2 = q->H2;
            r.VT = q->VT;
            r.c = q->theta + q->oc;
            r.l2 = q->d_l2;
            r.fpos = q->d_fpos;
            r.n2 = (int)q->l2.size();
            r.states = d_states;
            r.n = (int)n;
            r.b0 = (int)b0;
            r.nb = nb;
            r.h = q->h;
            r.H = q->H;
            r.logq = d_logq + b0;
            e = launch_wide_replay(r, s);
        } else {
            e = launch_logq(q->L, d_states, n, b0, q->d_fpos, q->h, nb, q->D, d_logq + b0, s);
        }
        if (e != hipSuccess) return hip_error(e, wide ? "logit replay" : "logq");
    }
    return PBIT_OK;
}

pbit_status pbit_proposal_sample_score(pbit_proposal q, uint32_t n, uint32_t chain_begin, uint64_t seed,
                                       uint32_t step, uint32_t *d_out, double *d_logq, const uint32_t *d_cur,
                                       double *d_logq_cur, void *hip_stream) {
    if (!q || !d_out || !d_logq || !d_cur || !d_logq_cur) return set_error(PBIT_E_INVALID_ARG, "NULL argument");
    if (n == 0) return PBIT_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    SampleArgs probe;
    std::memset(&probe, 0, sizeof(probe));
    probe.H = q->H;
    probe.h = q->h;
    probe.W = q->W;
    probe.D = q->D;
    probe.DP = q->DP;
    if (made_sample_dual_ok(probe))
        return sample_or_score(q, n, chain_begin, seed, step, d_out, d_logq, d_cur, s, d_logq_cur);
    pbit_status st = pbit_proposal_sample(q, n, chain_begin, seed, step, d_out, d_logq, s);
    if (st != PBIT_OK) return st;
    return pbit_proposal_score(q, d_cur, n, d_logq_cur, s);
}

}  // extern "C"

namespace {

// pbit_mh_run; with no_alloc (pbit_mh_run_static) the proposals and their
// log q live in the device's static scratch and the Gibbs sweeps take the
// generic kernels, so nothing is allocated or compiled.
pbit_status mh_run_impl(pbit_circuit c, pbit_proposal q, const pbit_mh_cfg *cfg, uint32_t *d_state, uint32_t *d_hist,
                        uint64_t *d_accepts, void *hip_stream, bool no_alloc) {
    if (!c || !q || !cfg || !d_state || !d_hist) return set_error(PBIT_E_INVALID_ARG, "NULL argument");
    if (q->circ != c) return set_error(PBIT_E_INVALID_ARG, "proposal belongs to another circuit handle");
    if (cfg->init != PBIT_INIT_ZERO && cfg->init != PBIT_INIT_RESUME) return set_error(PBIT_E_INVALID_ARG, "bad init");
    const uint64_t n = cfg->chains;
    if (n == 0) return PBIT_OK;
    if ((uint64_t)cfg->chain_begin + n > 0x100000000ull) return set_error(PBIT_E_INVALID_ARG, "chain index overflow");
    const uint64_t per_chain = (uint64_t)cfg->cycles * (1 + cfg->gibbs_per_mh);
    if (n * per_chain > 0xFFFFFFFFull) return set_error(PBIT_E_COUNT_OVERFLOW, "chains x transitions >= 2^32");
    if ((uint64_t)cfg->step_offset + cfg->cycles > 0xFFFFFFFFull ||
        (uint64_t)cfg->sweep_offset + (uint64_t)cfg->cycles * cfg->gibbs_per_mh > 0xFFFFFFFFull)
        return set_error(PBIT_E_INVALID_ARG, "step or sweep counter would wrap");
    // the state buffer holds only this circuit's chains, which the Gibbs
    // sweeps can address only on a single-circuit handle
    if (cfg->gibbs_per_mh && c->circuits.size() != 1)
        return set_error(PBIT_E_INVALID_ARG, "MH with Gibbs sweeps runs on single-circuit handles");
    hipStream_t s = (hipStream_t)hip_stream;
    uint32_t *prop = nullptr;
    double *lq_cur = nullptr, *lq_prop = nullptr;
    pbit_status st;
    if (no_alloc) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_error(e, "hipGetDevice");
        if (!q->theta || dev != q->dev)
            return set_error(PBIT_E_INVALID_ARG, "the proposal was set up on another device");
        const size_t b_prop = ((size_t)n * q->W * sizeof(uint32_t) + 255) & ~(size_t)255;
        const size_t b_lq = ((size_t)n * sizeof(double) + 255) & ~(size_t)255;
        if (b_prop + 2 * b_lq > MH_STATIC_BYTES)
            return set_error(PBIT_E_TOO_LARGE, "chains x (4 W + 16) bytes exceed the 16 MiB static MH scratch");
        void *base = nullptr;
        if ((st = static_scratch(dev, &base)) != PBIT_OK) return st;
        prop = (uint32_t *)base;
        lq_cur = (double *)((unsigned char *)base + b_prop);
        lq_prop = (double *)((unsigned char *)base + b_prop + b_lq);
    }
    if ((st = upload(q, s)) != PBIT_OK) return st;
    if ((st = refresh(q, s)) != PBIT_OK) return st;
    if (!no_alloc) {
        if (q->mh_cap < n) {
            q->prop = q->arena.alloc<uint32_t>((size_t)n * q->W);
            q->lq_cur = q->arena.alloc<double>(n);
            q->lq_prop = q->arena.alloc<double>(n);
            if (!q->prop || !q->lq_cur || !q->lq_prop) return set_error(PBIT_E_OOM, "MH workspace");
            q->mh_cap = (uint32_t)n;
        }
        prop = q->prop;
        lq_cur = q->lq_cur;
        lq_prop = q->lq_prop;
    }
    const uint32_t *dblob = nullptr;
    {
        std::lock_guard<std::mutex> lock(c->mu);
        if ((st = device_blobs(c, &dblob, no_alloc)) != PBIT_OK) return st;
    }
    const uint32_t *blob = dblob + c->blob_off[q->idx];
    const CompiledCircuit &k = c->circuits[q->idx];
    hipError_t e;
    if (cfg->init == PBIT_INIT_ZERO) {
        const int64_t tot = (int64_t)n * k.W;
        hipLaunchKernelGGL(fill_const_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, blob, d_state,
                           (int)n, (int)k.W);
        if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "fill");
    }
    std::vector<uint32_t> chains(c->circuits.size(), 0u);
    chains[q->idx] = (uint32_t)n;
    for (uint32_t cy = 0; cy < cfg->cycles; ++cy) {
        const uint32_t step = cfg->step_offset + cy;
        // every proposal and both log q are written before they are read:
        // nothing of the scratch needs clearing
        if ((st = pbit_proposal_sample_score(q, (uint32_t)n, cfg->chain_begin, cfg->seed, step, prop, lq_prop, d_state,
                                             lq_cur, s)) != PBIT_OK)
            return st;
        MhArgs a;
        std::memset(&a, 0, sizeof(a));
        a.blob = blob;
        a.state = d_state;
        a.prop = prop;
        a.logq_cur = lq_cur;
        a.logq_prop = lq_prop;
        a.accepts = (unsigned long long *)d_accepts;
        a.hist = d_hist + c->hist_off[q->idx];
        a.n = (int)n;
        a.W = (int)k.W;
        a.chain_begin = cfg->chain_begin;
        a.step = step;
        a.seed_lo = (uint32_t)cfg->seed;
        a.seed_hi = (uint32_t)(cfg->seed >> 32);
        a.hist_bins = 1u << (k.n + k.K);
        if (!cfg->gibbs_per_mh) {
            if ((e = launch_mh_accept(k.WS, a, s)) != hipSuccess) return hip_error(e, "mh accept");
        } else {
            // the sweeps' run takes the accept first (inside the first sweep
            // launch when that is the specialised kernel, else on its own)
            pbit_gibbs_cfg g;
            std::memset(&g, 0, sizeof(g));
            g.chains = chains.data();
            g.chain_begin = cfg->chain_begin;
            g.burn_in = 0;
            g.sweeps = cfg->gibbs_per_mh;
            g.seed = cfg->seed;
            g.sweep_offset = cfg->sweep_offset + cy * cfg->gibbs_per_mh;
            g.init = PBIT_INIT_RESUME;
            if ((st = run_gibbs(c, &g, d_state, d_hist, s, no_alloc, &a, q->idx)) != PBIT_OK) return st;
        }
    }
    return PBIT_OK;
}

}  // namespace

extern "C" {

pbit_status pbit_mh_run(pbit_circuit c, pbit_proposal q, const pbit_mh_cfg *cfg, uint32_t *d_state, uint32_t *d_hist,
                        uint64_t *d_accepts, void *hip_stream) {
    return mh_run_impl(c, q, cfg, d_state, d_hist, d_accepts, hip_stream, false);
}

pbit_status pbit_mh_run_static(pbit_circuit c, pbit_proposal q, const pbit_mh_cfg *cfg, uint32_t *d_state,
                               uint32_t *d_hist, uint64_t *d_accepts, void *hip_stream) {
    return mh_run_impl(c, q, cfg, d_state, d_hist, d_accepts, hip_stream, true);
}

pbit_status pbit_log_eval(const double *d_x, double *d_y, uint64_t n, void *hip_stream) {
    if (!d_x || !d_y) return set_error(PBIT_E_INVALID_ARG, "NULL argument");
    if (n >= (1ull << 40)) return set_error(PBIT_E_INVALID_ARG, "n must be below 2^40");
    hipError_t e = launch_log_eval(d_x, d_y, n, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_error(e, "log eval");
    return PBIT_OK;
}

pbit_status pbit_path_observables(pbit_circuit c, uint32_t idx, const uint32_t *d_state, uint32_t chains,
                                  uint32_t *d_bin, double *d_logmag, void *hip_stream) {
    if (!c || !d_state) return set_error(PBIT_E_INVALID_ARG, "NULL handle or d_state");
    if (idx >= c->circuits.size()) return set_error(PBIT_E_INVALID_ARG, "circuit index out of range");
    if (chains > 0x7FFFFFFFu) return set_error(PBIT_E_INVALID_ARG, "chains must be below 2^31");
    if (chains == 0 || (!d_bin && !d_logmag)) return PBIT_OK;
    const uint32_t *dblob = nullptr;
    pbit_status st;
    {
        std::lock_guard<std::mutex> lock(c->mu);
        if ((st = device_blobs(c, &dblob)) != PBIT_OK) return st;
    }
    const CompiledCircuit &k = c->circuits[idx];
    hipError_t e = launch_observe(k.WS, dblob + c->blob_off[idx], d_state, (int)chains, d_bin, d_logmag,
                                  (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_error(e, "path observables");
    return PBIT_OK;
}

}  // extern "C"
