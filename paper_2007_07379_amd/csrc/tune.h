// Launch-shape choice for the Gibbs kernels (internal).
#pragma once
#include <cstdint>

#include "../../include/pbit.h"
#include "compile.h"
#include "runtime.h"

namespace pbit {

struct TuneChoice {
    uint32_t block = 256;     // chains per workgroup
    uint64_t group = 0;       // sweeps per launch
    bool lds_hist = true;     // histogram privatised in LDS
    bool tog = true;          // LDS toggle tables (else per-bit cone toggles)
    bool pair = false;        // two lanes per chain (uniform circuits)
    bool jit = false;         // circuit-specialised kernel (uniform circuits)
    uint32_t lanes_log2 = 0;  // specialised kernel: log2(lanes per chain)
    bool path_hist = false;   // specialised kernel: LDS counts per path, binned at the end
    bool keys = false;        // specialised kernel: bins stored as keys, counted by the key histogram
    bool general = false;     // specialised kernel of a circuit with other conditionals (pbit_general_sweep)
};

// Kind of the specialised kernel (JitHist in jit.h): the histogram placement,
// with JIT_PAIRED (4) for the two-wave form of pbit_general_sweep.
inline uint32_t jit_hist_kind(const TuneChoice &t) {
    return (t.path_hist ? 2u : (t.keys ? 3u : (t.lds_hist ? 1u : 0u))) | (t.general && t.lanes_log2 ? 4u : 0u);
}

// Is a circuit-specialised kernel of this histogram kind (any kind) for
// circuit i compiled in the handle for the current device?  The handle's
// mutex must be held.
bool jit_compiled(pbit_circuit c, uint32_t i, uint32_t kind);
bool jit_compiled_any(pbit_circuit c, uint32_t i);

// Explicit cfg fields win; unset ones come from the autotuned table of the
// handle (if pbit_autotune ran or loaded a cache) or from the static rules.
TuneChoice tune_choice(pbit_circuit c, uint32_t i, uint32_t chains, uint64_t total_sweeps,
                       const pbit_gibbs_cfg *cfg);

struct BatchTuning {
    uint32_t wg_per_cu[3];
    size_t hist_lds_max;
};
BatchTuning tune_batch(pbit_circuit c, const pbit_gibbs_cfg *cfg);

}  // namespace pbit
