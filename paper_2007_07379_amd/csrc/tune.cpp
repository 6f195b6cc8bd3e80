// Launch-shape choice: explicit cfg fields, then the handle's autotuned
// table, then static rules.
#include "tune.h"

#include <algorithm>

#include "blob.h"
#include "gibbs.h"
#include "jit.h"
#include "keyhist.h"

namespace pbit {

TuneChoice tune_choice(pbit_circuit c, uint32_t i, uint32_t chains, uint64_t total_sweeps,
                       const pbit_gibbs_cfg *cfg) {
    const CompiledCircuit &k = c->circuits[i];
    TuneChoice t;
    constexpr size_t LDS_MAX = 160 * 1024;
    const size_t hist_bytes = ((size_t)1 << (k.n + k.K)) * 4;
    // static rules: toggle tables when they leave room; the histogram
    // privatised in LDS when it fits next to them and the threshold tables;
    // small workgroups when a short run would not fill 256 CUs
    t.tog = gibbs_lds_bytes(k.blob.data(), true, false) <= 96 * 1024;
    t.lds_hist = gibbs_lds_bytes(k.blob.data(), t.tog, true) <= LDS_MAX;
    t.block = 256;
    if (chains < 256u * 256u && hist_bytes <= 32 * 1024) t.block = 64;
    // two lanes per chain when the chains alone would leave SIMDs with a
    // single wave (256 CUs x 4 SIMDs x 64 lanes = 65,536 chains)
    t.pair = k.uniform && chains <= 98304u && gibbs_pair_lds_bytes(k.blob.data(), false) <= 96 * 1024;
    auto it = c->tuned.find(i);
    const bool tuned = it != c->tuned.end();
    if (tuned) {
        t.block = it->second.block;
        t.lds_hist = it->second.lds_hist;
        t.tog = it->second.tog;
        t.pair = it->second.pair;
    }
    if (cfg->lanes_per_chain == 1) t.pair = false;
    if (cfg->lanes_per_chain == 2) t.pair = k.uniform;
    // three-qubit products need the whole lattice in one lane, rebuilt each
    // sweep from the toggle tables
    if (k.ny) {
        t.pair = false;
        t.tog = true;
    }
    if (cfg->toggle_mode == 1) t.tog = true;
    if (cfg->toggle_mode == 2) t.tog = false;
    if (cfg->hist_mode == 1) t.lds_hist = true;
    if (cfg->hist_mode == 2) t.lds_hist = false;
    if (t.lds_hist && gibbs_lds_bytes(k.blob.data(), t.tog, true) > LDS_MAX) t.tog = false;
    if (t.lds_hist && gibbs_lds_bytes(k.blob.data(), t.tog, true) > LDS_MAX && cfg->hist_mode != 1)
        t.lds_hist = false;
    // the pair kernel always stages its own split toggle tables
    if (t.pair && cfg->toggle_mode == 2) t.pair = false;
    if (t.pair) {
        t.tog = true;
        if (!tuned || !it->second.pair) {
            t.lds_hist = gibbs_pair_lds_bytes(k.blob.data(), true) <= LDS_MAX;
            t.block = 512;  // 256 chains
        }
        if (cfg->hist_mode == 1) t.lds_hist = true;
        if (cfg->hist_mode == 2) t.lds_hist = false;
        if (cfg->block_size) t.block = 2 * cfg->block_size;
    } else if (cfg->block_size) {
        t.block = cfg->block_size;
    } else if (t.block > 256) {
        t.block = 256;  // a tuned pair shape, overridden to one lane per chain
    }
    t.group = total_sweeps;
    if (cfg->sweeps_per_launch) t.group = std::min<uint64_t>(cfg->sweeps_per_launch, total_sweeps);

    // circuit-specialised kernel: runs of 2^33 updates or more (the run-time
    // compile takes about a second), or any run once the kernel it needs is
    // already compiled in the handle (an earlier long run paid for it),
    // unless the caller asks for a generic toggle mode
    const uint64_t work = (uint64_t)chains * total_sweeps * k.h;
    const bool auto_rule = cfg->specialize == 0 && cfg->toggle_mode == 0;
    const bool short_run = work < (1ull << 33);
    t.jit = cfg->specialize == 2 || (auto_rule && (!short_run || jit_compiled_any(c, i)));
    if (t.jit && !k.uniform) {
        // other conditionals: sweeps depend on each other, so one lane per
        // chain, or two waves per 64 chains (splitting each colour's bits)
        // for runs of at most 32,768 chains, which leave most SIMDs without
        // a wave (measured on rctch12: 10 % faster there, 27 % slower at
        // 65,536 chains, where the barriers and the doubled cone XORs cost
        // more than the second wave per SIMD gains), or when lanes_per_chain
        // asks for more than one; threshold tables and the histogram in LDS
        // when they fit
        const uint32_t L = cfg->lanes_per_chain;
        t.general = true;
        t.lanes_log2 = (L >= 2 || (L == 0 && chains <= 32768u)) ? 1u : 0u;
        t.pair = false;
        t.tog = true;
        t.path_hist = t.keys = false;
        const size_t thr_b = (size_t)k.blob[H_THR_TOTAL] * 4;
        const size_t hist_b = ((size_t)1 << (k.n + k.K)) * 4;
        const size_t flips_b = t.lanes_log2 ? jit_general_lds_bytes(k, false, 256, true) -
                                                  jit_general_lds_bytes(k, false, 256, false)
                                            : 0;
        t.lds_hist = cfg->hist_mode == 1 || (cfg->hist_mode != 2 && thr_b + hist_b + flips_b <= LDS_MAX);
        t.block = cfg->block_size ? cfg->block_size : 256;
        if (t.lanes_log2 && t.block % 128) t.block = t.block < 128 ? 128 : 256;  // pairs of waves
    } else if (t.jit) {
        uint32_t L = cfg->lanes_per_chain;
        if (!L) {
            // enough lanes for four waves per SIMD, each lane keeping >= 16 sweeps
            L = 1;
            while (L < 8 && (uint64_t)chains * L < 4ull * 65536 && t.group / (2 * L) >= 16) L *= 2;
        }
        t.lanes_log2 = L >= 8 ? 3 : (L >= 4 ? 2 : (L >= 2 ? 1 : 0));
        t.pair = false;
        t.tog = true;
        const size_t hist_b = ((size_t)1 << (k.n + k.K)) * 4;
        const size_t rows_b = jit_rows_bytes(k);
        const bool lds_fits = rows_b + hist_b <= LDS_MAX;
        const bool path_fits = k.h <= 16 && rows_b + ((size_t)4 << k.h) <= LDS_MAX;
        const uint32_t bits = k.n + k.K;
        const bool keys_ok = bits <= KEYHIST_MAX_BITS && chains <= (1u << 24);
        const uint64_t per_wg = (uint64_t)1024 * t.group >> t.lanes_log2;
        // Keys pay when HBM atomics would bound the sweep: the chip retires
        // about 27e9 of them a second when the bins are spread (fewer when
        // they are not), i.e. 37 ps a sample, while a sample costs about
        // (34 + 6) lane-ops per Philox block and 8 per lattice word, at 85 %
        // of 39.3e12 lane-ops/s, plus about 4 ps of key histogram (16 bytes
        // of HBM traffic a key and the partial rows).
        const double ps_sample = (40.0 * ((k.h + 3) / 4) + 8.0 * k.W) / (39.3 * 0.85);
        const bool keys_pay = ps_sample + 4.0 < 37.0;
        // automatic choice, in this order: counts per path when the paths are
        // few next to the samples of a workgroup (at least 16 per path: a
        // sweep then skips the lattice, phase and bin, and the histogram sees
        // one atomic per path that occurred); the histogram in LDS when it
        // fits; bins stored as keys when that pays; else HBM atomics
        t.lds_hist = t.path_hist = t.keys = false;
        if (k.h <= 14 && path_fits && per_wg >= (16ull << k.h))
            t.path_hist = true;
        else if (lds_fits)
            t.lds_hist = true;
        else if (keys_ok && keys_pay)
            t.keys = true;
        if (cfg->hist_mode == 1 || cfg->hist_mode == 2 || (cfg->hist_mode == 3 && path_fits) ||
            (cfg->hist_mode == 4 && keys_ok)) {
            t.lds_hist = cfg->hist_mode == 1;
            t.path_hist = cfg->hist_mode == 3;
            t.keys = cfg->hist_mode == 4;
        }
        t.block = t.lds_hist || t.path_hist ? 1024 : 256;
        if (cfg->block_size) t.block = cfg->block_size;
    }
    if (t.jit && auto_rule && short_run && !jit_compiled(c, i, jit_hist_kind(t))) {
        // a short run does not pay for compiling another kind: generic kernels
        pbit_gibbs_cfg g = *cfg;
        g.specialize = 1;
        return tune_choice(c, i, chains, total_sweeps, &g);
    }
    return t;
}

bool jit_compiled(pbit_circuit c, uint32_t i, uint32_t kind) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    return c->jit.count(std::make_tuple(dev, i, kind)) != 0;
}

bool jit_compiled_any(pbit_circuit c, uint32_t i) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    // histogram kinds 0..3, each also with JIT_PAIRED
    for (uint32_t kind = 0; kind < 8; ++kind)
        if (c->jit.count(std::make_tuple(dev, i, kind))) return true;
    return false;
}

BatchTuning tune_batch(pbit_circuit c, const pbit_gibbs_cfg *cfg) {
    (void)cfg;
    BatchTuning b;
    for (int i = 0; i < 3; ++i) b.wg_per_cu[i] = c->tuned_batch.wg_per_cu[i];
    b.hist_lds_max = c->tuned_batch.hist_lds_max;
    return b;
}

}  // namespace pbit
