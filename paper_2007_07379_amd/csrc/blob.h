// Device image of one compiled circuit: a flat uint32 array read by the
// sampling kernels with wave-uniform (scalar) loads.
//
// Header words (index into the blob):
#pragma once
#include <stdint.h>

namespace pbit {

constexpr uint32_t BLOB_MAGIC = 0x70626974u;  // "pbit"
constexpr int MAX_W = 32;          // lattice words (1024 lattice bits)
constexpr int MAX_FW = 8;          // free-bit words (256 free bits)
constexpr int MAX_K = 8;           // phase bits
constexpr int MAX_SCOPE = 12;      // neighbourhood bits of one threshold table
constexpr int MAX_QD = 64;         // distinct quadratic phase offsets
constexpr int MAX_N = 24;          // qubits (histogram 2^(n+K) bins)

enum Header : uint32_t {
    H_MAGIC = 0,
    H_N,
    H_D,
    H_K,
    H_W,
    H_H,          // free bits h
    H_L,          // lattice bits n (d+1)
    H_CID,        // circuit id (< 2^16)
    H_NCOL,       // colours
    H_UNIFORM,    // 1 if every threshold is 2^31
    H_AWORD,      // output state alpha = bits [d n, d n + n): word ...
    H_ASHIFT,     // ... and shift
    H_PCONST,     // constant term of the phase polynomial (mod 2^K)
    H_LINMASK,    // bit t set if linear plane t is nonzero
    H_NQD,        // number of quadratic offsets
    H_FW,         // ceil(h / 32)
    H_OFF_CONST,  // WS words: lattice with every free bit 0
    H_OFF_FPOS,   // h words: lattice index of free bit b
    H_OFF_CONE,   // h * WS words: cone mask of free bit b
    H_OFF_LIN,    // K * WS words: linear phase planes
    H_OFF_QD,     // NQD records of qd_stride(K, WS) words
    H_OFF_COLIDX, // NCOL * MAX_FW pairs (offset, count) into the entry list
    H_OFF_COLENT, // entries (j << 4 | mask): Philox block j, bits 4j+t with mask bit t
    H_OFF_THRINFO,// h records of THR_STRIDE words: table offset, scope size, positions
    H_OFF_THRTAB, // thresholds, uint32
    H_THR_TOTAL,  // number of threshold entries
    H_HBITS,      // n + K
    H_TOTAL,      // blob length in words
    H_WS,         // storage stride of per-word arrays (a compiled kernel width >= W)
    H_NBLK,       // Philox blocks per sweep: ceil(h / 4)
    H_TOGW,       // row stride of the toggle tables: WS rounded up to a multiple of 4
    H_OFF_TOG,    // NBLK * 16 * TOGW words: XOR of the cones of each subset of a block's bits
    H_NQG,        // merged quadratic groups (see below)
    H_OFF_QG,     // NQG group records
    H_NRE,        // gates with non-constant magnitude (real-energy records)
    H_OFF_RE,     // NRE records of RE_STRIDE words
    H_NY,         // derived AND variables of three-qubit permutation gates
    H_OFF_Y,      // NY records of Y_STRIDE words, in layer order
    H_NSOFT,      // gates with soft zeros
    H_OFF_SOFT,   // NSOFT records of SOFT_STRIDE words
    H_COUNT = 48  // header words (must exceed every index above)
};

// Lattice widths with a compiled sampling kernel; a circuit of W words runs
// on the smallest listed width >= W and its image is padded to that stride.
constexpr uint32_t KERNEL_WIDTHS[] = {1, 2, 3, 4, 6, 8, 10, 12, 13, 14, 16, 17, 20, 24, 28, 32};
constexpr inline uint32_t kernel_words(uint32_t W) {
    for (uint32_t v : KERNEL_WIDTHS)
        if (W <= v) return v;
    return 0;
}

constexpr int THR_STRIDE = 2 + MAX_SCOPE;
// threshold tables up to this many words are staged in LDS; larger ones are
// read from the image in device memory
constexpr uint32_t THR_LDS_MAX_WORDS = 16384;
// real-energy record: [0] arity a, [1..2] input lattice bits, [3..4] output
// lattice bits, [5..7] unused, then 16 doubles (as 32 words): ln |U[out][in]|
// at index out * 2^a + in (0 where the entry is zero).
constexpr int RE_STRIDE = 8 + 32;
constexpr inline uint32_t qd_stride(uint32_t K, uint32_t W) { return 2 + K * W; }
// derived AND variable: [0], [1] = lattice bits (previous layer) whose AND it
// is, then WS words: the lattice bits whose form contains it
constexpr inline uint32_t y_stride(uint32_t WS) { return 2 + WS; }
// gate with soft zeros: [0], [1] input lattice bits, [2], [3] output lattice
// bits, [4] mask: bit o * 4 + i set where the entry (out o, in i) is a soft
// zero (one-qubit gates use bits 0 and 2 as i0 and o0; the others never
// set); a sample whose lattice meets one is not binned
constexpr uint32_t SOFT_STRIDE = 5;
// quadratic record: [0] = offset delta (1..63), [1] = mask of nonzero planes,
// then K planes of WS words: bit i of plane t set if bit t of the coefficient
// of x_i x_{i+delta} is set.
//
// merged quadratic group: [0] = plane t, [1] = m, then m entries of
// (delta, WS mask words).  The masks of one group are pairwise disjoint, so
// sum_delta popcount(x & (x >> delta) & mask_delta)
//   = popcount(x & OR_delta((x >> delta) & mask_delta))
// and the group costs one funnel shift and one three-input bit op per word
// per delta plus one AND and one popcount per word.
constexpr inline uint32_t qg_entry_stride(uint32_t WS) { return 1 + WS; }

}  // namespace pbit

namespace pbit {
static_assert(H_OFF_RE < H_COUNT, "blob header overflows H_COUNT");
}
