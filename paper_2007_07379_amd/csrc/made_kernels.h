// Device helpers and launch interfaces of the MADE / MH kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "made.h"
#include "made_log_table.h"

namespace pbit {

// The proposal's probability of a 1 at a free position, as the uint32
// threshold the sampler compares its Philox draw with: P(1) = T / 2^32
// exactly, whatever rounding produced T.  The sigmoid is evaluated in FP32
// (the logit is FP32 already) with the hardware exponential and reciprocal
// (each within about one ulp); scaling by 2^32 is exact and the conversion
// truncates.  T is kept in [1, 2^32 - 1] (a NaN logit gives 1) so every path
// has q > 0.  The samplers and the scorers call this same function, so all
// of them see the same T.
__device__ __forceinline__ uint32_t made_threshold(float logit) {
    const float p = __builtin_amdgcn_rcpf(1.0f + __expf(-logit));
    const float t = p * 4294967296.0f;
    return t >= 4294967296.0f ? 0xFFFFFFFFu : (t >= 1.0f ? (uint32_t)t : 1u);
}

// Natural logarithm of a positive normal double, within one ulp (0.74 ulp
// at worst over 3.3e4 arguments, the 2^32 grid of the thresholds and edge
// cases, emulated exactly on the host; the GPU test bounds it against numpy
// over 10^6).  x = 2^e m, m in [1, 2); the top 8 fraction bits j select an
// inverse G_j of 9 significant bits with |m G_j - 1| <= 2^-8, so that
// r = m G_j - 1 is exact in one fma, and log x = (e + k_j) log 2 + T_j +
// log1p(r) with T_j = -log G_j - k_j log 2 (k_j = 1 above sqrt(2), so that
// the bins next to 1 have T = 0 and results near 0 keep their relative
// accuracy).  log 2 and T_j are split so that (e + k_j) log2_hi + T_hi is
// exact; log1p(r) - r is r^2 times a degree-6 polynomial (the next term is
// below 2^-67 |r|).  About 13 FP64 operations and three table reads
// (made_log_table.h, written by gen_log_table.py).
__device__ __forceinline__ double made_log(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t hw = (uint32_t)(b >> 32);
    const int e = (int)(hw >> 20) - 1023;
    const int j = (int)((hw >> 12) & 255u);
    const double m = __longlong_as_double((long long)((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    const double r = fma(m, MADE_LOG_G[j], -1.0);  // exact
    const double E = (double)(e + MADE_LOG_K[j]);
    double q = -0.125;
    q = fma(q, r, 1.0 / 7.0);
    q = fma(q, r, -1.0 / 6.0);
    q = fma(q, r, 0.2);
    q = fma(q, r, -0.25);
    q = fma(q, r, 1.0 / 3.0);
    q = fma(q, r, -0.5);
    const double r2 = r * r;
    const double lo = fma(r2, q, fma(E, MADE_LOG_LN2_LO, MADE_LOG_TL[j]));
    const double hi = fma(E, MADE_LOG_LN2_HI, MADE_LOG_TH[j]);  // exact
    return hi + (r + lo);
}

// log of the probability of `bit` under threshold T: log(T / 2^32) for a 1,
// log((2^32 - T) / 2^32) for a 0 (the scaling by 2^-32 is exact).  The
// argument is selected first, so a wave whose lanes hold both values
// evaluates one logarithm, not two.  Every sampler and scorer sums these
// same values.
__device__ __forceinline__ double made_log_prob(uint32_t T, uint32_t bit) {
    const double v = bit ? (double)T : 4294967296.0 - (double)T;
    return made_log(v * 0x1p-32);
}

struct SampleArgs {
    const uint32_t *blob;  // circuit image (cones, constant lattice, circuit id)
    const bf16 *W1T, *W2T, *VT;
    const float *b1, *b2, *c;
    const int4 *phase;    // per free bit: first-layer unit range, second-layer unit range
    const int4 *phase_k;  // per free bit: K ends of the three products, lattice position
    const uint32_t *sched;  // per free bit: 16 words (unit ranges, half tiles, K chunks, position, cone)
    int n, h, W, D, DP, H;
    uint32_t chain_begin, step, seed_lo, seed_hi;
    uint32_t *out;        // word-major lattice words of the proposals (may be NULL)
    double *logq;         // log q of each proposal (score mode: of each scored path)
    double *logq_cur;     // dual mode: log q of the scored current paths
    const uint32_t *score;  // score mode: word-major paths whose bits are read instead of drawn
    int defer;            // set by the launcher: 0 logs in the loop, 1/2 deferred (2: over the activations)
    // the wide register-resident sampler's schedule: per free bit {first
    // step, end step, lattice position p, 0}; per step {layer (0 or 1),
    // first unit of the half tile, K chunks, for layer 2 the phase's units
    // [lo, hi) of the half tile as lo | hi << 8}; per free bit its cone
    // words (cone_stride apart, at least 16 of them, zero past W)
    const int4 *wphase, *wstep;
    const uint32_t *wcone;
    int cone_stride, nsteps;
};

// The distance between consecutive free bits' cones in SampleArgs::wcone
// for W lattice words.
inline uint32_t wd_cone_stride(uint32_t W) { return W < 16 ? 16 : W; }

hipError_t launch_made_sample(const SampleArgs &a, hipStream_t s);
// True if one of the samplers can run the shape of a (n, h, W, D, DP, H set):
// the register-resident kernel, or made_sample_kernel within 160 KiB of LDS.
bool made_sample_launchable(const SampleArgs &a);
// True if the wide register-resident sampler takes the shape of a (networks
// of 256 < H <= 1024, lattices of at most 512 bits, at most 128 free bits);
// its scorer is then the GEMMs and launch_wide_replay.
bool made_sample_wide_ok(const SampleArgs &a);
// The scorer's logits and log q for the networks of the wide sampler
// (made_sample_wide_ok), from the batch's second-layer activations: paths
// b0 .. b0 + nb - 1 of `states` (word-major, n paths a word), H2 row i =
// path b0 + i, log q into logq[0 .. nb).  l2: the sampler's layer-2 steps
// in order, {first unit of the half tile, lo | hi << 8}; fpos: the lattice
// position of each free bit.
struct ReplayArgs {
    const bf16 *H2, *VT;
    const float *c;
    const int2 *l2;
    const int *fpos;
    const uint32_t *states;
    int n, b0, nb, h, H, n2;
    double *logq;
};
hipError_t launch_wide_replay(const ReplayArgs &a, hipStream_t s);
// One pass that draws proposals (out, logq) and scores the paths in `score`
// (logq_cur) with the arithmetic of the two separate calls; only for the
// networks made_sample_dual_ok accepts (H <= 256, lattices <= 256 bits).
bool made_sample_dual_ok(const SampleArgs &a);
hipError_t launch_made_sample_dual(const SampleArgs &a, hipStream_t s);
hipError_t launch_unpack(const uint32_t *states, int n, int D, int DP, bf16 *X, hipStream_t s);
// y[i] = made_log(x[i]) for i < n (n < 2^40)
hipError_t launch_log_eval(const double *x, double *y, uint64_t n, hipStream_t s);
// bf16 shadow Wb (K x N, row-major) and transpose WT (N x KP, zero-padded)
// of an fp32 K x N weight W; one launch for `count` (1 to 3) weights.
struct ShadowJob {
    const float *W;
    int K, N, KP;
    bf16 *Wb, *WT;
};
// The parameter gradient from the training GEMMs' leftovers and, with adam,
// one Adam step (grad_final_kernel, adam_shadow_kernel).  Flat parameter order W1 [D][H],
// b1, W2 [H][H], b2, V [H][D], c at the given offsets.  With adam and
// sh[0].Wb set, the step also writes the bf16 shadows of the updated W1, W2
// and V (sh[0..2], W unused), in place of a separate shadow launch.
struct GradFinal {
    int adam;
    float *th, *m, *v;  // Adam state (adam)
    float *grad;        // gradient out (!adam)
    float lr, b1, b2, eps, c1, c2;
    int64_t P, oW1, ob1, oW2, ob2, oV, oc;
    int D, H;
    const float *pW1, *pW2, *pV;  // split-K slices of the weight gradients
    int zW1, zW2, zV;             // their slice counts (>= 1)
    const float *cb1, *cb2, *cc;  // 64-row column partials of G1, G2, G3
    int chunks;                   // their row-chunk count
    const int *deg_in, *deg1, *deg2, *deg_out;
    const float *losspart;        // loss shares, nloss of them, summed into *loss (may be NULL)
    int nloss;
    float *loss;
    ShadowJob sh[3];              // shadows of W1, W2, V written by the Adam step (sh[0].Wb NULL: none)
    // With the shadows: rows [ux_b0, ux_b0 + ux_n) of a word-major state
    // array (row stride ux_stride) unpacked into ux_X [ux_n][ux_DP] bf16 in
    // the same launch (the next training batch; ux_n = 0: none)
    const uint32_t *ux_states;
    uint64_t ux_stride, ux_b0;
    int ux_n, ux_DP;
    bf16 *ux_X;
};
// Thread e < n DP / 8 of an unpack of rows [b0, b0 + n) of a word-major
// state array (row stride `stride`): X[b][8g .. 8g + 7] = the path's bits
// 8g .. 8g + 7 as bf16 0 / 1 (positions >= D as 0), one 16-byte store, so a
// wave's stores run along the rows (b = e / (DP / 8), g = e % (DP / 8); DP a
// multiple of 32).
__device__ __forceinline__ void unpack_row8(const uint32_t *__restrict__ states, uint64_t stride, uint64_t b0,
                                            int D, int DP, bf16 *__restrict__ X, uint32_t e) {
    const uint32_t G = (uint32_t)DP >> 3;
    const uint32_t b = e / G, g = e - b * G;
    const int i0 = (int)g * 8, left = D - i0;
    uint32_t bits = 0;
    if (left > 0) {
        bits = (states[(uint64_t)(i0 >> 5) * stride + b0 + b] >> (i0 & 31)) & 0xFFu;
        if (left < 8) bits &= (1u << left) - 1u;
    }
    constexpr uint32_t ONE = 0x3F80u;  // bf16 1.0
    uint4 w;
    w.x = ((bits & 1u) ? ONE : 0u) | ((bits & 2u) ? ONE << 16 : 0u);
    w.y = ((bits & 4u) ? ONE : 0u) | ((bits & 8u) ? ONE << 16 : 0u);
    w.z = ((bits & 16u) ? ONE : 0u) | ((bits & 32u) ? ONE << 16 : 0u);
    w.w = ((bits & 64u) ? ONE : 0u) | ((bits & 128u) ? ONE << 16 : 0u);
    *reinterpret_cast<uint4 *>(X + (uint64_t)b * DP + i0) = w;
}
hipError_t launch_grad_final(const GradFinal &a, hipStream_t s);
// G[m][j] = 0 where A[m][j] <= 0 (n x N bf16, row-major, N % 8 == 0), and
// the 64-row column partials of the gated G into colpart (ceil(n / 64) x N).
hipError_t launch_gate_colsum(bf16 *G, const bf16 *A, int n, int N, float *colpart, hipStream_t s);
struct ShadowJobs {
    ShadowJob j[3];
};
hipError_t launch_shadow(const ShadowJobs &jobs, int count, hipStream_t s);
hipError_t launch_logq(const float *L, const uint32_t *states, uint64_t stride, uint64_t b0, const int *fpos, int h,
                       int n, int D, double *out, hipStream_t s);

// Metropolis-Hastings accept of independence proposals (mh.hip).
struct MhArgs {
    const uint32_t *blob;
    uint32_t *state;          // word-major current lattices, updated in place
    const uint32_t *prop;     // word-major proposals
    const double *logq_cur, *logq_prop;
    unsigned long long *accepts;  // per-chain accept counters (may be NULL)
    uint32_t *hist;           // bins the post-transition state (may be NULL)
    int n, W;
    uint32_t chain_begin, step, seed_lo, seed_hi;
    uint32_t hist_bins;       // 2^(n+K); privatised in LDS per workgroup when small
};
hipError_t launch_mh_accept(uint32_t Wk, const MhArgs &a, hipStream_t s);
// Per-path bin and ln|psi| (non-constant-magnitude gates) of n word-major
// lattices; bin or logmag may be NULL.
hipError_t launch_observe(uint32_t Wk, const uint32_t *blob, const uint32_t *state, int n, uint32_t *bin,
                          double *logmag, hipStream_t s);

}  // namespace pbit
