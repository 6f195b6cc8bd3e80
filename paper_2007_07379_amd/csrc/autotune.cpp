// Autotuner: times candidate launch shapes on short runs of the caller's
// workload and keeps the fastest in the handle (and optionally a JSON-lines
// cache file keyed by a hash of the compiled circuits and chain counts).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pbit.h"
#include "blob.h"
#include "gibbs.h"
#include "runtime.h"

namespace pbit {
namespace {

uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

std::string hex64(uint64_t v) {
    char buf[32];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)v);
    return buf;
}

bool load_cache(pbit_circuit c, const char *path, const std::string &key) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[1 << 16];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (!std::strstr(line, ("\"key\": \"" + key + "\"").c_str())) continue;
        const char *b = std::strstr(line, "\"batch\": [");
        unsigned w0, w1, w2, hm;
        if (!b || std::sscanf(b, "\"batch\": [%u, %u, %u, %u]", &w0, &w1, &w2, &hm) != 4) continue;
        c->tuned_batch.wg_per_cu[0] = w0;
        c->tuned_batch.wg_per_cu[1] = w1;
        c->tuned_batch.wg_per_cu[2] = w2;
        c->tuned_batch.hist_lds_max = hm;
        c->tuned.clear();
        const char *s = std::strstr(line, "\"single\": [");
        if (s) {
            s += std::strlen("\"single\": [");
            unsigned i, blk, lh, tg, pr;
            int used = 0;
            while (std::sscanf(s, " [%u, %u, %u, %u, %u]%n", &i, &blk, &lh, &tg, &pr, &used) == 5) {
                TunedSingle t;
                t.block = blk;
                t.lds_hist = lh != 0;
                t.tog = tg != 0;
                t.pair = pr != 0;
                c->tuned[i] = t;
                s += used;
                while (*s == ',' || *s == ' ') ++s;
            }
        }
        found = true;
    }
    std::fclose(f);
    return found;
}

void save_cache(pbit_circuit c, const char *path, const std::string &key) {
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"batch\": [%u, %u, %u, %u], \"single\": [", key.c_str(),
                 c->tuned_batch.wg_per_cu[0], c->tuned_batch.wg_per_cu[1], c->tuned_batch.wg_per_cu[2],
                 c->tuned_batch.hist_lds_max);
    bool first = true;
    for (auto &kv : c->tuned) {
        std::fprintf(f, "%s[%u, %u, %u, %u, %u]", first ? "" : ", ", kv.first, kv.second.block,
                     kv.second.lds_hist ? 1u : 0u, kv.second.tog ? 1u : 0u, kv.second.pair ? 1u : 0u);
        first = false;
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
}

}  // namespace
}  // namespace pbit

using namespace pbit;

extern "C" pbit_status pbit_autotune(pbit_circuit c, const pbit_gibbs_cfg *cfg, const char *cache_path,
                                     void *hip_stream) {
    if (!c || !cfg || !cfg->chains) return set_error(PBIT_E_INVALID_ARG, "NULL handle or cfg");
    const uint32_t nc = (uint32_t)c->circuits.size();
    uint64_t h = 0xCBF29CE484222325ull;
    for (auto &k : c->circuits) h = fnv1a(h, k.blob.data(), k.blob.size() * sizeof(uint32_t));
    h = fnv1a(h, cfg->chains, nc * sizeof(uint32_t));
    const std::string key = hex64(h);
    if (cache_path && load_cache(c, cache_path, key)) {
        c->tune_epoch++;
        return PBIT_OK;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    uint64_t state_words = 0;
    for (uint32_t i = 0; i < nc; ++i) state_words += (uint64_t)cfg->chains[i] * c->circuits[i].W;
    uint32_t *d_state = nullptr, *d_hist = nullptr;
    hipError_t e = hipMalloc(&d_state, std::max<uint64_t>(state_words, 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&d_hist, std::max<uint64_t>(c->hist_total, 1) * 4);
    if (e != hipSuccess) {
        if (d_state) (void)hipFree(d_state);
        return set_error(PBIT_E_OOM, "autotune buffers");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        (void)hipFree(d_state);
        (void)hipFree(d_hist);
        return hip_error(e, "autotune events");
    }
    const uint32_t trial = (uint32_t)std::max<uint64_t>(8, std::min<uint64_t>(64, (uint64_t)cfg->burn_in + cfg->sweeps));
    pbit_status status = PBIT_OK;
    // time one configuration: one warm-up run, then the best of two
    auto time_cfg = [&](const pbit_gibbs_cfg &t, float *ms) -> pbit_status {
        float best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            hipError_t ee = hipEventRecord(e0, s);
            if (ee != hipSuccess) return hip_error(ee, "autotune event");
            pbit_status st = run_gibbs(c, &t, d_state, d_hist, s);
            if (st != PBIT_OK) return st;
            if ((ee = hipEventRecord(e1, s)) == hipSuccess) ee = hipEventSynchronize(e1);
            if (ee != hipSuccess) return hip_error(ee, "autotune sync");
            float v = 0;
            if ((ee = hipEventElapsedTime(&v, e0, e1)) != hipSuccess) return hip_error(ee, "autotune timing");
            if (r > 0) best = std::min(best, v);
        }
        *ms = best;
        return PBIT_OK;
    };
    pbit_gibbs_cfg base = *cfg;
    base.burn_in = 0;
    base.sweeps = trial;
    base.init = PBIT_INIT_ZERO;
    base.use_graph = 0;
    base.sweeps_per_launch = 0;
    const bool persistent = cfg->persistent == 1 || (cfg->persistent == 0 && nc > 1);
    c->tuned.clear();
    c->tune_epoch++;
    if (persistent) {
        // persistent grid size and LDS histogram threshold
        float best = 1e30f;
        TunedBatch bestb = c->tuned_batch;
        for (uint32_t hm : {0u, 16u * 1024u, 64u * 1024u}) {
            for (uint32_t wg : {1u, 2u, 3u, 4u, 6u, 8u}) {
                c->tuned_batch.hist_lds_max = hm;
                for (int k = 0; k < 3; ++k) c->tuned_batch.wg_per_cu[k] = wg;
                pbit_gibbs_cfg t = base;
                t.wg_per_cu = 0;
                float ms = 0;
                if ((status = time_cfg(t, &ms)) != PBIT_OK) goto done;
                if (ms < best) {
                    best = ms;
                    bestb = c->tuned_batch;
                }
            }
        }
        c->tuned_batch = bestb;
    }
    // single-circuit launches: workgroup size, histogram privatisation,
    // toggle tables
    for (uint32_t i = 0; i < nc; ++i) {
        if (!cfg->chains[i]) continue;
        const CompiledCircuit &k = c->circuits[i];
        if (persistent && k.uniform) continue;  // runs in the persistent launch
        std::vector<uint32_t> only(nc, 0u);
        only[i] = cfg->chains[i];
        float best = 1e30f;
        TunedSingle bt;
        for (uint32_t lanes : {1u, 2u}) {
            if (lanes == 2 && !k.uniform) continue;
        for (uint32_t tog : {1u, 2u}) {
            if (lanes == 2 && tog == 2) continue;
            if (tog == 1 && gibbs_lds_bytes(k.blob.data(), true, false) > 96 * 1024) continue;
            for (uint32_t hmode : {1u, 2u}) {
                if (hmode == 1 && gibbs_lds_bytes(k.blob.data(), tog == 1, true) > 160 * 1024) continue;
                for (uint32_t blk : {64u, 128u, 256u}) {
                    pbit_gibbs_cfg t = base;
                    t.chains = only.data();
                    t.persistent = 2;
                    t.block_size = blk;
                    t.hist_mode = hmode;
                    t.toggle_mode = tog;
                    t.lanes_per_chain = lanes;
                    float ms = 0;
                    if ((status = time_cfg(t, &ms)) != PBIT_OK) goto done;
                    if (ms < best) {
                        best = ms;
                        bt.block = lanes == 2 ? 2 * blk : blk;
                        bt.lds_hist = hmode == 1;
                        bt.tog = tog == 1;
                        bt.pair = lanes == 2;
                    }
                }
            }
        }
        }
        c->tuned[i] = bt;
    }
    c->tune_epoch++;
    if (cache_path) save_cache(c, cache_path, key);
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_state);
    (void)hipFree(d_hist);
    return status;
}
