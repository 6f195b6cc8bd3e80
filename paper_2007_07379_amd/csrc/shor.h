// Period finding by column sampling (internal launch interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbit {

// Keys the preparation sorts: T rounded up to a power of two, at least 4.
uint32_t shor_pad(uint32_t T);

// Draws T first-register configurations, sorts (f << 32 | x) into keys
// (shor_pad(T) words; the first T are the samples sorted by f, then x) and
// writes P[k] for k < 2^n.  N < 2^31, n <= 30.
hipError_t launch_shor(uint64_t N, uint64_t a, uint32_t n, uint32_t T, uint64_t seed, float *P, uint64_t *keys,
                       hipStream_t s);

}  // namespace pbit
