// Run planning for pbit_gibbs_run: device images, sweep groups, histogram
// privatisation choice, optional hipGraph capture and replay of the sweep
// groups.
#include "runtime.h"

#include <algorithm>
#include <cstring>

#include "blob.h"
#include "gibbs.h"
#include "tune.h"

pbit_circuit_s::~pbit_circuit_s() {
    for (auto &kv : graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    for (auto *m : {&blobs, &scratch, &work})
        for (auto &kv : *m)
            if (kv.second.ptr) (void)hipFree(kv.second.ptr);
}

namespace pbit {

namespace {

constexpr size_t LDS_LIMIT = 160 * 1024;

pbit_status ensure_buf(std::map<int, DevBuf> &m, int dev, size_t bytes, void **out) {
    DevBuf &b = m[dev];
    if (b.bytes < bytes) {
        if (b.ptr) {
            hipError_t e = hipFree(b.ptr);
            if (e != hipSuccess) return hip_error(e, "hipFree");
        }
        b.ptr = nullptr;
        b.bytes = 0;
        hipError_t e = hipMalloc(&b.ptr, bytes);
        if (e != hipSuccess) return set_error(PBIT_E_OOM, "hipMalloc of library scratch failed");
        b.bytes = bytes;
    }
    *out = b.ptr;
    return PBIT_OK;
}

}  // namespace

pbit_status device_blobs(pbit_circuit c, const uint32_t **base) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    auto it = c->blobs.find(dev);
    if (it == c->blobs.end() || !it->second.ptr) {
        std::vector<uint32_t> all;
        c->blob_off.clear();
        for (auto &k : c->circuits) {
            c->blob_off.push_back(all.size());
            all.insert(all.end(), k.blob.begin(), k.blob.end());
        }
        void *p = nullptr;
        pbit_status st = ensure_buf(c->blobs, dev, all.size() * sizeof(uint32_t), &p);
        if (st != PBIT_OK) return st;
        e = hipMemcpy(p, all.data(), all.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_error(e, "hipMemcpy of circuit images");
    }
    *base = (const uint32_t *)c->blobs[dev].ptr;
    return PBIT_OK;
}

pbit_status run_gibbs(pbit_circuit c, const pbit_gibbs_cfg *cfg, uint32_t *d_state, uint32_t *d_hist,
                      hipStream_t stream) {
    if (!c || !cfg || !cfg->chains) return set_error(PBIT_E_INVALID_ARG, "NULL handle, cfg or chains");
    if (!d_hist) return set_error(PBIT_E_INVALID_ARG, "d_hist is NULL");
    if (cfg->init != PBIT_INIT_ZERO && cfg->init != PBIT_INIT_RESUME)
        return set_error(PBIT_E_INVALID_ARG, "bad init mode");
    if (cfg->init == PBIT_INIT_RESUME && !d_state) return set_error(PBIT_E_INVALID_ARG, "RESUME needs d_state");
    if (cfg->hist_mode > 2) return set_error(PBIT_E_INVALID_ARG, "bad hist_mode");
    if (cfg->toggle_mode > 2) return set_error(PBIT_E_INVALID_ARG, "bad toggle_mode");
    if (cfg->block_size && (cfg->block_size % 64 || cfg->block_size > 256))
        return set_error(PBIT_E_INVALID_ARG, "block_size must be a multiple of 64 in 64..256");
    const uint64_t total = (uint64_t)cfg->burn_in + cfg->sweeps;
    if ((uint64_t)cfg->sweep_offset + total > 0xFFFFFFFFull)
        return set_error(PBIT_E_INVALID_ARG, "sweep counter would wrap");
    if (cfg->use_graph && !stream) return set_error(PBIT_E_INVALID_ARG, "graph replay needs a non-null stream");
    const uint32_t nc = (uint32_t)c->circuits.size();
    uint64_t state_words = 0;
    for (uint32_t i = 0; i < nc; ++i) {
        const uint64_t ch = cfg->chains[i];
        if ((uint64_t)cfg->chain_begin + ch > 0x100000000ull)
            return set_error(PBIT_E_INVALID_ARG, "chain index would exceed 2^32");
        if (ch * (uint64_t)cfg->sweeps > 0xFFFFFFFFull)
            return set_error(PBIT_E_COUNT_OVERFLOW, "chains x sweeps >= 2^32 for circuit " + std::to_string(i));
        state_words += ch * c->circuits[i].W;
    }
    if (total == 0) return PBIT_OK;

    std::lock_guard<std::mutex> lock(c->mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    const uint32_t *dblob = nullptr;
    pbit_status st = device_blobs(c, &dblob);
    if (st != PBIT_OK) return st;

    // plan every launch first (argument errors before any enqueue)
    struct Plan {
        GibbsLaunch a;
        uint32_t Wk;
        bool uniform;
        bool tog;
        uint32_t block;
        size_t lds;
    };
    std::vector<Plan> plans;
    uint32_t *state_base = d_state;
    bool need_scratch = false;
    std::vector<TuneChoice> choices(nc);
    for (uint32_t i = 0; i < nc; ++i) {
        if (!cfg->chains[i]) continue;
        choices[i] = tune_choice(c->circuits[i], cfg->chains[i], total, cfg);
        if (!d_state && choices[i].group < total) need_scratch = true;
    }
    if (need_scratch) {
        void *p = nullptr;
        st = ensure_buf(c->scratch, dev, std::max<uint64_t>(state_words, 1) * sizeof(uint32_t), &p);
        if (st != PBIT_OK) return st;
        state_base = (uint32_t *)p;
    }
    uint64_t soff = 0;
    for (uint32_t i = 0; i < nc; ++i) {
        const CompiledCircuit &k = c->circuits[i];
        const uint32_t ch = cfg->chains[i];
        if (!ch) continue;
        const TuneChoice &tc = choices[i];
        const size_t thr_bytes = k.uniform ? 0 : (size_t)k.blob[H_THR_TOTAL] * sizeof(uint32_t);
        if (thr_bytes > 64 * 1024) return set_error(PBIT_E_TOO_LARGE, "threshold tables exceed 64 KiB of LDS");
        const bool lds_hist = tc.lds_hist;
        const size_t lds = gibbs_lds_bytes(k.blob.data(), tc.tog, lds_hist);
        if (lds > LDS_LIMIT) return set_error(PBIT_E_INVALID_ARG, "LDS-privatised histogram does not fit");
        uint32_t *sp = state_base ? state_base + soff : nullptr;
        for (uint64_t done = 0; done < total; done += tc.group) {
            Plan p;
            std::memset(&p.a, 0, sizeof(p.a));
            p.a.blob = dblob + c->blob_off[i];
            p.a.state = sp;
            p.a.hist = d_hist + c->hist_off[i];
            p.a.n_chains = ch;
            p.a.chain_begin = cfg->chain_begin;
            p.a.seed_lo = (uint32_t)cfg->seed;
            p.a.seed_hi = (uint32_t)(cfg->seed >> 32);
            p.a.sweep_begin = (uint32_t)(cfg->sweep_offset + done);
            p.a.n_sweeps = (uint32_t)std::min<uint64_t>(tc.group, total - done);
            p.a.bin_from = cfg->sweep_offset + cfg->burn_in;
            p.a.resume = done > 0 ? 1u : (cfg->init == PBIT_INIT_RESUME ? 1u : 0u);
            p.a.lds_hist = lds_hist ? 1u : 0u;
            p.Wk = k.WS;
            p.uniform = k.uniform;
            p.tog = tc.tog;
            p.block = tc.block;
            p.lds = lds;
            plans.push_back(p);
        }
        soff += (uint64_t)ch * k.W;
    }

    auto enqueue = [&]() -> pbit_status {
        for (const Plan &p : plans) {
            hipError_t le = launch_gibbs(p.Wk, p.uniform, p.tog, p.a, p.block, p.lds, stream);
            if (le != hipSuccess) return hip_error(le, "gibbs kernel launch");
        }
        return PBIT_OK;
    };

    if (!cfg->use_graph) return enqueue();

    // graph replay keyed by everything that shapes the captured launches
    std::vector<uint64_t> key = {(uint64_t)(uintptr_t)stream, (uint64_t)(uintptr_t)d_state,
                                 (uint64_t)(uintptr_t)d_hist, (uint64_t)(uintptr_t)state_base,
                                 cfg->chain_begin, cfg->burn_in, cfg->sweeps, cfg->seed, cfg->sweep_offset,
                                 cfg->init, cfg->sweeps_per_launch, cfg->block_size, cfg->hist_mode,
                                 cfg->toggle_mode};
    for (uint32_t i = 0; i < nc; ++i) key.push_back(cfg->chains[i]);
    GraphCache &gc = c->graphs[dev];
    if (!(gc.exec && gc.key == key)) {
        if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
        if (gc.graph) (void)hipGraphDestroy(gc.graph);
        gc.exec = nullptr;
        gc.graph = nullptr;
        e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
        st = enqueue();
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(stream, &g);
        if (st != PBIT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_error(e, "hipGraphInstantiate");
        }
        gc.graph = g;
        gc.key = key;
    }
    e = hipGraphLaunch(gc.exec, stream);
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
    return PBIT_OK;
}

}  // namespace pbit
