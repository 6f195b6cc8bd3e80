// Persistent batched launch interface (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbit {

// A circuit of the batch, as offsets (in 32-bit words) from the launch's
// base pointers, so the kernel derives its pointers from kernel arguments
// (known global memory, the image read with scalar loads).
struct BatchCirc {
    uint64_t blob_off;   // device image of the circuit in the image buffer
    uint64_t state_off;  // this circuit's word-major lattice words in the state buffer
    uint64_t hist_off;   // this circuit's histogram in the histogram buffer
    uint32_t n_chains;
    uint32_t lds_hist;   // histogram privatised in LDS for this circuit
    uint32_t Wk;         // compiled width (image stride)
    uint32_t pad;
};

struct BatchTile {
    uint32_t circ;  // index into the BatchCirc array
    uint32_t c0;    // first local chain of the tile
};

struct BatchArgs {
    const BatchCirc *circs;
    const BatchTile *tiles;
    uint32_t ntiles;
    uint32_t *queue;  // tile counter, reset before every launch
    uint32_t chain_begin, seed_lo, seed_hi;
    uint32_t sweep_begin, n_sweeps, bin_from, resume;
};

// lattice-width class of a circuit: 0 for W <= 8, 1 for W <= 17, 2 above
int batched_class_of(uint32_t Wk);
// blob_base: the images of all circuits; state_base (may be NULL: no state
// buffer) and hist_base: the buffers the circuits' offsets point into.
hipError_t launch_batched(int cls, const BatchArgs &a, const uint32_t *blob_base, uint32_t *state_base,
                          uint32_t *hist_base, uint32_t grid, size_t lds, hipStream_t s);

}  // namespace pbit
