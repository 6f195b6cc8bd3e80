// Period finding by column sampling (Sec. 5, Fig. 7).  A sample is a
// configuration x of the n-p-bit first register, drawn uniformly; its
// second-register value is f(x) = a^x mod N; the inverse-QFT column of x,
// 2^(-n/2) exp(-2 pi i k x / 2^n) over k, is added to column f(x) of psi,
// and the output law is the row sum of |psi|^2.  With T samples:
//
//   P[k] = 2^(-n) / T * sum over values f of |sum over sampled x with
//          f(x) = f of exp(-2 pi i k x / 2^n)|^2.
//
// shor_prepare_kernel (one workgroup) draws the x, evaluates f and sorts the
// pairs (f, x) so that equal f are adjacent (the grouping that keeps the
// memory at the samples plus one output row, instead of 2^n x 2^n);
// shor_column_kernel gives every lane one output k and walks the sorted
// samples, whose loads are uniform across the wave (scalar loads), so each
// term costs the lane one multiply, one conversion, one scale, a hardware
// cosine and sine and two adds.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "philox.h"
#include "shor.h"

namespace pbit {

namespace {

constexpr uint32_t PREP_THREADS = 1024;
constexpr uint32_t COL_THREADS = 256;
constexpr uint32_t TAG_SHOR = 3;
constexpr uint32_t SMALL_SORT = 1u << 16;  // keys one workgroup sorts

__device__ __forceinline__ uint64_t powmod(uint64_t a, uint64_t e, uint64_t N) {
    uint64_t r = 1 % N, b = a % N;  // N < 2^31: every product below 2^62
    while (e) {
        if (e & 1u) r = r * b % N;
        b = b * b % N;
        e >>= 1;
    }
    return r;
}

// Keys of Philox blocks b0, b0 + step, ... below Tpad / 4: (f << 32 | x),
// padding all ones.
__device__ __forceinline__ void draw_keys(uint64_t N, uint64_t a, uint32_t n, uint32_t T, uint32_t Tpad,
                                          uint32_t seed_lo, uint32_t seed_hi, uint64_t *__restrict__ keys,
                                          uint32_t b0, uint32_t step) {
    const uint32_t mask = (1u << n) - 1u;
    for (uint32_t b = b0; b < Tpad / 4; b += step) {
        const U4 u = philox4x32_10(b, 0u, 0u, TAG_SHOR << 16, seed_lo, seed_hi);
        const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
        for (uint32_t e = 0; e < 4; ++e) {
            const uint32_t i = 4 * b + e;
            uint64_t key = ~0ull;
            if (i < T) {
                const uint32_t x = w[e] & mask;
                key = (powmod(a, x, N) << 32) | x;
            }
            keys[i] = key;
        }
    }
}

// One compare-exchange of the bitonic network (sequence size `size`,
// distance `stride`) for pair index i < Tpad / 2.
__device__ __forceinline__ void bitonic_pair(uint64_t *__restrict__ keys, uint32_t i, uint32_t size,
                                             uint32_t stride) {
    const uint32_t lo = 2 * stride * (i / stride) + (i % stride);
    const uint32_t hi = lo + stride;
    const bool up = (lo & size) == 0;
    const uint64_t p = keys[lo], q = keys[hi];
    if ((p > q) == up) {
        keys[lo] = q;
        keys[hi] = p;
    }
}

// Small T: draws, f and the whole sort in one workgroup, a barrier between
// the steps of the network.
__global__ void __launch_bounds__(PREP_THREADS) shor_prepare_kernel(uint64_t N, uint64_t a, uint32_t n, uint32_t T,
                                                                   uint32_t Tpad, uint32_t seed_lo, uint32_t seed_hi,
                                                                   uint64_t *__restrict__ keys) {
    draw_keys(N, a, n, T, Tpad, seed_lo, seed_hi, keys, threadIdx.x, PREP_THREADS);
    __syncthreads();
    for (uint32_t size = 2; size <= Tpad; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < Tpad / 2; i += PREP_THREADS) bitonic_pair(keys, i, size, stride);
            __syncthreads();
        }
    }
}

// Large T: the draws over the whole grid, then one launch per step.
__global__ void __launch_bounds__(256) shor_draw_kernel(uint64_t N, uint64_t a, uint32_t n, uint32_t T,
                                                       uint32_t Tpad, uint32_t seed_lo, uint32_t seed_hi,
                                                       uint64_t *__restrict__ keys) {
    draw_keys(N, a, n, T, Tpad, seed_lo, seed_hi, keys, blockIdx.x * 256 + threadIdx.x, gridDim.x * 256);
}

__global__ void __launch_bounds__(256) shor_bitonic_kernel(uint64_t *__restrict__ keys, uint32_t Tpad,
                                                          uint32_t size, uint32_t stride) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < Tpad / 2) bitonic_pair(keys, i, size, stride);
}

// ks = k << (32 - n): the 32-bit product ks x is (k x mod 2^n) << (32 - n),
// so 2^-32 times it is the phase k x / 2^n mod 1 in revolutions, the unit of
// the hardware sine and cosine.
__device__ __forceinline__ void add_term(uint32_t ks, uint32_t x, float &sr, float &si) {
    const float u = (float)(ks * x) * 0x1p-32f;
    sr += __builtin_amdgcn_cosf(u);
    si -= __builtin_amdgcn_sinf(u);
}

__device__ __forceinline__ void step(uint64_t key, uint32_t ks, uint32_t &fprev, double &acc, float &sr, float &si) {
    const uint32_t f = (uint32_t)(key >> 32);
    if (f != fprev) {  // wave-uniform: the keys are the same for every lane
        acc += (double)sr * sr + (double)si * si;
        sr = 0.0f;
        si = 0.0f;
        fprev = f;
    }
    add_term(ks, (uint32_t)key, sr, si);
}

__global__ void __launch_bounds__(COL_THREADS) shor_column_kernel(const uint64_t *__restrict__ keys, uint32_t n,
                                                                 uint32_t T, double inv_T, double inv_2n,
                                                                 float *__restrict__ P) {
    const uint32_t k = blockIdx.x * COL_THREADS + threadIdx.x;
    const uint32_t mask = (1u << n) - 1u;
    const uint32_t ks = k << (32 - n);
    double acc = 0.0;
    float sr = 0.0f, si = 0.0f;
    uint32_t fprev = (uint32_t)(keys[0] >> 32);
    uint32_t i = 0;
    // eight keys per scalar load batch
    for (; i + 8 <= T; i += 8) {
        uint64_t kk[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) kk[e] = keys[i + e];
#pragma unroll
        for (int e = 0; e < 8; ++e) step(kk[e], ks, fprev, acc, sr, si);
    }
    for (; i < T; ++i) step(keys[i], ks, fprev, acc, sr, si);
    acc += (double)sr * sr + (double)si * si;
    if (k <= mask) P[k] = (float)(acc * inv_2n * inv_T);
}

}  // namespace

uint32_t shor_pad(uint32_t T) {
    uint32_t p = 4;
    while (p < T) p <<= 1;
    return p;
}

hipError_t launch_shor(uint64_t N, uint64_t a, uint32_t n, uint32_t T, uint64_t seed, float *P, uint64_t *keys,
                       hipStream_t s) {
    const uint32_t Tpad = shor_pad(T);
    hipError_t e;
    if (Tpad <= SMALL_SORT) {
        hipLaunchKernelGGL(shor_prepare_kernel, dim3(1), dim3(PREP_THREADS), 0, s, N, a, n, T, Tpad, (uint32_t)seed,
                           (uint32_t)(seed >> 32), keys);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        const uint32_t g = (Tpad / 2 + 255) / 256;
        hipLaunchKernelGGL(shor_draw_kernel, dim3((Tpad / 4 + 255) / 256), dim3(256), 0, s, N, a, n, T, Tpad,
                           (uint32_t)seed, (uint32_t)(seed >> 32), keys);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (uint32_t size = 2; size <= Tpad; size <<= 1)
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                hipLaunchKernelGGL(shor_bitonic_kernel, dim3(g), dim3(256), 0, s, keys, Tpad, size, stride);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
    }
    const uint32_t grid = (uint32_t)(((1ull << n) + COL_THREADS - 1) / COL_THREADS);
    hipLaunchKernelGGL(shor_column_kernel, dim3(grid), dim3(COL_THREADS), 0, s, (const uint64_t *)keys, n, T,
                       1.0 / (double)T, 1.0 / (double)(1ull << n), P);
    return hipGetLastError();
}

}  // namespace pbit
