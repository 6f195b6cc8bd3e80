// Deferred binning: histogram of a stream of 32-bit bin keys (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pbit {

// Largest histogram (log2 of the bin count) the key histogram serves: up to
// 2^(bits - 15) buckets of 2^15 LDS bins.
constexpr uint32_t KEYHIST_MAX_BITS = 24;
constexpr uint32_t KEYHIST_MAX_BUCKETS = 1u << (KEYHIST_MAX_BITS - 15);
// Most keys one call counts (offsets inside the scratch are 32-bit).
constexpr uint64_t KEYHIST_MAX_KEYS = 1ull << 30;
// Upper bound of the partial rows (2^bits words each).
constexpr uint64_t KEYHIST_PART_BYTES = 256ull << 20;

// Device scratch one call needs for M keys below 2^bits.
size_t keyhist_scratch_bytes(uint64_t M, uint32_t bits);

// hist[key] += 1 for each of the M keys (all below 2^bits; larger keys are
// not counted).  keys must be 16-byte aligned, scratch 256-byte aligned
// with keyhist_scratch_bytes(M, bits) bytes.  Enqueues six kernels on s.
hipError_t launch_keyhist(const uint32_t *keys, uint64_t M, uint32_t bits, void *scratch, uint32_t *hist,
                          hipStream_t s);

}  // namespace pbit
