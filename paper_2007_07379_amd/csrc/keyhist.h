// Deferred binning: histogram of a stream of 32-bit bin keys (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pbit {

// Largest histogram (log2 of the bin count) the key histogram serves: up to
// 2^(bits - 15) buckets of 2^15 LDS bins, each reading every key.
constexpr uint32_t KEYHIST_MAX_BITS = 22;
// Upper bound of the partial rows (one per slab, 2^bits words each).
constexpr uint64_t KEYHIST_PART_BYTES = 256ull << 20;

struct KeyhistShape {
    uint32_t S = 0;        // slabs (a multiple of 8)
    uint32_t grid = 0;     // workgroups: S x buckets
    uint64_t slab = 0;     // keys per slab (a multiple of 4)
    size_t part_bytes = 0; // bytes of the partial rows
};
KeyhistShape keyhist_shape(uint64_t M, uint32_t bits);

// hist[key] += 1 for each of the M keys (all below 2^bits).  keys must be
// 16-byte aligned; part holds keyhist_shape(M, bits).part_bytes.  Keys of
// 2^bits or more are not counted.  Enqueues two kernels on s.
hipError_t launch_keyhist(const uint32_t *keys, uint64_t M, uint32_t bits, uint32_t *part, uint32_t *hist,
                          hipStream_t s);

}  // namespace pbit
