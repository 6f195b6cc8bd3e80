// Launch-shape rules for the Gibbs kernels.
#include "tune.h"

#include <algorithm>

#include "blob.h"
#include "gibbs.h"

namespace pbit {

TuneChoice tune_choice(const CompiledCircuit &k, uint32_t chains, uint64_t total_sweeps,
                       const pbit_gibbs_cfg *cfg) {
    TuneChoice t;
    constexpr size_t LDS_MAX = 160 * 1024;
    const size_t hist_bytes = ((size_t)1 << (k.n + k.K)) * 4;
    // toggle tables when they leave room; the histogram privatised in LDS
    // when it fits next to them and the threshold tables
    t.tog = gibbs_lds_bytes(k.blob.data(), true, false) <= 96 * 1024;
    if (cfg->toggle_mode == 1) t.tog = true;
    if (cfg->toggle_mode == 2) t.tog = false;
    t.lds_hist = gibbs_lds_bytes(k.blob.data(), t.tog, true) <= LDS_MAX;
    if (cfg->hist_mode == 1) t.lds_hist = true;
    if (cfg->hist_mode == 2) t.lds_hist = false;
    if (t.lds_hist && gibbs_lds_bytes(k.blob.data(), t.tog, true) > LDS_MAX) t.tog = false;
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
