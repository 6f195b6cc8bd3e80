// Launch-shape choice for the Gibbs kernels (internal).
#pragma once
#include <cstdint>

#include "../../include/pbit.h"
#include "compile.h"

namespace pbit {

struct TuneChoice {
    uint32_t block = 256;     // chains per workgroup
    uint64_t group = 0;       // sweeps per launch
    bool lds_hist = true;     // histogram privatised in LDS
    bool tog = true;          // LDS toggle tables (else per-bit cone toggles)
};

// Explicit cfg fields win; unset ones come from the tuning table (if one was
// loaded or measured for this circuit class) or from the static rules.
TuneChoice tune_choice(const CompiledCircuit &k, uint32_t chains, uint64_t total_sweeps,
                       const pbit_gibbs_cfg *cfg);

}  // namespace pbit
