// Launch-shape rules for the Gibbs kernels.
#include "tune.h"

#include <algorithm>

#include "blob.h"

namespace pbit {

TuneChoice tune_choice(const CompiledCircuit &k, uint32_t chains, uint64_t total_sweeps,
                       const pbit_gibbs_cfg *cfg) {
    TuneChoice t;
    const size_t thr_bytes = (size_t)k.blob[H_THR_TOTAL] * 4;
    const size_t hist_bytes = ((size_t)1 << (k.n + k.K)) * 4;
    // LDS privatisation when the histogram fits next to the threshold tables
    t.lds_hist = thr_bytes + hist_bytes <= 160 * 1024;
    if (cfg->hist_mode == 1) t.lds_hist = true;
    if (cfg->hist_mode == 2) t.lds_hist = false;
    // one workgroup per CU when a large histogram occupies the LDS; smaller
    // groups otherwise so that short runs still spread over 256 CUs
    t.block = 256;
    if (chains < 256u * 256u && hist_bytes <= 32 * 1024) t.block = 64;
    if (cfg->block_size) t.block = cfg->block_size;
    t.group = total_sweeps;
    if (cfg->sweeps_per_launch) t.group = std::min<uint64_t>(cfg->sweeps_per_launch, total_sweeps);
    return t;
}

}  // namespace pbit
