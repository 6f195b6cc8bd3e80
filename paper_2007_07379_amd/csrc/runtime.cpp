// Run planning for pbit_gibbs_run: device images, sweep groups, histogram
// privatisation choice, optional hipGraph capture and replay of the sweep
// groups.
#include "runtime.h"

#include <algorithm>
#include <cstring>

#include "batched.h"
#include "blob.h"
#include "gibbs.h"
#include "keyhist.h"
#include "made_kernels.h"
#include "tune.h"

pbit_circuit_s::~pbit_circuit_s() {
    for (auto &kv : graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    for (auto *m : {&blobs, &scratch, &work, &keys, &keypart})
        for (auto &kv : *m)
            if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    for (auto &kv : jit)
        if (kv.second.module) (void)hipModuleUnload(kv.second.module);
    for (hipModule_t m : jit_groups) (void)hipModuleUnload(m);
    for (auto &kv : side) {
        for (int k = 0; k < pbit::SIDE_STREAMS; ++k) {
            if (kv.second.s[k]) (void)hipStreamDestroy(kv.second.s[k]);
            if (kv.second.join[k]) (void)hipEventDestroy(kv.second.join[k]);
        }
        if (kv.second.fork) (void)hipEventDestroy(kv.second.fork);
    }
}

namespace pbit {

namespace {

constexpr size_t LDS_LIMIT = 160 * 1024;
// keys of one launch of a specialised kernel that stores its bins as keys
// (1 GiB of key buffer)
constexpr uint64_t KEYS_MAX = 1ull << 28;

pbit_status ensure_side(std::map<int, SideStreams> &m, int dev, SideStreams **out) {
    SideStreams &ss = m[dev];
    if (!ss.fork) {
        for (int k = 0; k < SIDE_STREAMS; ++k) {
            hipError_t e = hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ss.join[k], hipEventDisableTiming);
            if (e != hipSuccess) return hip_error(e, "side stream creation");
        }
        hipError_t e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming);
        if (e != hipSuccess) return hip_error(e, "side stream creation");
    }
    *out = &ss;
    return PBIT_OK;
}

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

pbit_status device_blobs(pbit_circuit c, const uint32_t **base, bool no_alloc) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    auto it = c->blobs.find(dev);
    if (it == c->blobs.end() || !it->second.ptr) {
        if (no_alloc) return set_error(PBIT_E_INVALID_ARG, "circuit images are not resident on this device");
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

bool batchable(pbit_circuit c, uint32_t i, const pbit_gibbs_cfg *cfg) {
    const uint32_t nc = (uint32_t)c->circuits.size();
    const bool persistent = cfg->persistent == 1 || (cfg->persistent == 0 && nc > 1);
    const CompiledCircuit &k = c->circuits[i];
    return persistent && k.uniform && gibbs_lds_bytes(k.blob.data(), true, false) <= 64 * 1024 &&
           cfg->toggle_mode != 2;
}

// With specialize == 2 the circuits of a persistent batch with at least
// BATCH_SPEC_CHAINS chains leave the batch for launches of their own
// circuit-specialised kernel (each costs a run-time compile, at most
// BATCH_SPEC_MAX of them, the heaviest by chains x free bits first); the
// persistent launch keeps the many small circuits.  With specialize == 0
// (auto) the same happens when the whole run is long (2^33 updates or more:
// the compiles run on host threads at once, about a second for a hundred
// kernels, and are kept in the handle); otherwise only a circuit whose run
// alone pays for its compile (2^33 updates, the single-circuit rule) leaves.
// (The 256-circuit batch of 2^22 chains: 0.736 of the VALU peak with a
// threshold of 1,024 chains, 0.754 with 512, 0.73 with 256.)
constexpr uint32_t BATCH_SPEC_CHAINS = 512;
constexpr size_t BATCH_SPEC_MAX = 256;
std::vector<bool> batch_specialised(pbit_circuit c, const pbit_gibbs_cfg *cfg) {
    const uint32_t nc = (uint32_t)c->circuits.size();
    std::vector<bool> out(nc, false);
    if (cfg->specialize == 1 || (cfg->specialize == 0 && cfg->toggle_mode != 0)) return out;
    const uint64_t total = (uint64_t)cfg->burn_in + cfg->sweeps;
    uint64_t run_updates = 0;
    for (uint32_t i = 0; i < nc; ++i) run_updates += (uint64_t)cfg->chains[i] * total * c->circuits[i].h;
    const bool long_run = run_updates >= (1ull << 33);
    std::vector<std::pair<uint64_t, uint32_t>> cand;
    for (uint32_t i = 0; i < nc; ++i) {
        if (cfg->chains[i] < BATCH_SPEC_CHAINS || !batchable(c, i, cfg)) continue;
        if (cfg->specialize == 0 && !long_run && (uint64_t)cfg->chains[i] * total * c->circuits[i].h < (1ull << 33))
            continue;
        cand.push_back({(uint64_t)cfg->chains[i] * c->circuits[i].h, i});
    }
    std::stable_sort(cand.begin(), cand.end(), [](const std::pair<uint64_t, uint32_t> &a,
                                                  const std::pair<uint64_t, uint32_t> &b) { return a.first > b.first; });
    for (size_t r = 0; r < cand.size() && r < BATCH_SPEC_MAX; ++r) out[cand[r].second] = true;
    return out;
}

bool runs_batched(pbit_circuit c, uint32_t i, const pbit_gibbs_cfg *cfg, const std::vector<bool> &spec) {
    return batchable(c, i, cfg) && !spec[i];
}

// Launch shape of circuit i outside the persistent launch: a circuit that
// left a batch to be specialised (batch_specialised) takes its specialised
// kernel under the automatic rule too.
TuneChoice member_choice(pbit_circuit c, uint32_t i, const pbit_gibbs_cfg *cfg, uint64_t total,
                         const std::vector<bool> &spec) {
    if (spec[i] && cfg->specialize == 0) {
        pbit_gibbs_cfg g = *cfg;
        g.specialize = 2;
        return tune_choice(c, i, cfg->chains[i], total, &g);
    }
    return tune_choice(c, i, cfg->chains[i], total, cfg);
}

// Builds the circuit-specialised kernels a run needs that the handle does not
// hold (nor has failed to build): one workgroup per CU holds an LDS histogram,
// so such a kernel gets 1024 threads (four waves per SIMD) unless that spills
// registers, then 512; without it, 256-thread workgroups.  Each round
// compiles the current candidate of every pending kernel (equal sources are
// compiled once per process) and loads them; a kernel that spills moves on
// to its next candidate, keeping the spilling one if that fails.  Failures are recorded
// in jit_failed (the run then takes the generic kernels, or reports them).
// hipRTC compiles one program at a time per process, so a round's kernels
// go into one program (about a quarter of the time of separate programs).
void compile_jits(pbit_circuit c, int dev, const pbit_gibbs_cfg *cfg, const std::vector<TuneChoice> &choices,
                  const std::vector<bool> &batched) {
    struct Need {
        uint32_t i, kind;
        std::vector<uint32_t> mbs;
        size_t cand = 0;
        JitKernel best;  // a loaded kernel that spills, kept until a better one loads
        JitSource src;
        std::string log;
    };
    std::vector<Need> need;
    const uint32_t nc = (uint32_t)c->circuits.size();
    for (uint32_t i = 0; i < nc; ++i) {
        if (!cfg->chains[i] || batched[i] || !choices[i].jit) continue;
        const uint32_t kind = jit_hist_kind(choices[i]);
        const auto key = std::make_tuple(dev, i, kind);
        if (c->jit.count(key) || c->jit_failed.count(key)) continue;
        bool dup = false;
        for (const Need &n : need) dup |= n.i == i && n.kind == kind;
        if (dup) continue;
        Need n;
        n.i = i;
        n.kind = kind;
        const bool lds = c->circuits[i].uniform && (kind == JIT_HIST_LDS || kind == JIT_HIST_PATHS);
        n.mbs = lds ? std::vector<uint32_t>{1024, 512} : std::vector<uint32_t>{256};
        need.push_back(std::move(n));
    }
    if (need.empty()) return;
    auto finish = [&](Need &n) {
        const auto key = std::make_tuple(dev, n.i, n.kind);
        if (n.best.fn) {
            n.best.hist_kind = n.kind;
            c->jit.emplace(key, n.best);
        } else {
            c->jit_failed[key] = n.log.empty() ? std::string("no kernel") : n.log;
        }
    };
    std::vector<Need *> pending;
    for (Need &n : need) pending.push_back(&n);
    while (!pending.empty()) {
        std::vector<Need *> round;
        std::vector<const JitSource *> srcs;
        for (Need *n : pending) {
            n->src = jit_uniform_source(c->circuits[n->i], n->kind, n->mbs[n->cand]);
            if (n->src.lds_bytes > JIT_LDS_LIMIT) {
                n->log = "LDS of the specialised kernel exceeds 160 KiB";
                finish(*n);
                continue;
            }
            round.push_back(n);
            srcs.push_back(&n->src);
        }
        // the round as one program; if that fails, each kernel on its own
        // (so one failure costs only its own kernel)
        std::vector<JitKernel> built(round.size());
        std::vector<bool> ok(round.size(), false);
        hipModule_t gm = nullptr;
        std::string glog;
        if (round.size() > 1 && jit_build_group(srcs, &gm, &built, &glog)) {
            c->jit_groups.push_back(gm);
            ok.assign(round.size(), true);
        } else {
            for (size_t j = 0; j < round.size(); ++j) ok[j] = jit_build(round[j]->src, &built[j], &round[j]->log);
        }
        pending.clear();
        for (size_t j = 0; j < round.size(); ++j) {
            Need &n = *round[j];
            if (ok[j]) {
                if (n.best.module) (void)hipModuleUnload(n.best.module);
                n.best = built[j];
            }
            const bool spills = n.best.fn && n.best.scratch_bytes != 0;
            if (spills && ok[j] && n.cand + 1 < n.mbs.size()) {
                n.cand += 1;
                pending.push_back(&n);
            } else {
                finish(n);
            }
        }
    }
}

pbit_status run_gibbs(pbit_circuit c, const pbit_gibbs_cfg *cfg_in, uint32_t *d_state, uint32_t *d_hist,
                      hipStream_t stream, bool no_alloc, const MhArgs *mh, uint32_t mh_circ) {
    if (!c || !cfg_in || !cfg_in->chains) return set_error(PBIT_E_INVALID_ARG, "NULL handle, cfg or chains");
    pbit_gibbs_cfg cfg_na;
    const pbit_gibbs_cfg *cfg = cfg_in;
    if (no_alloc) {
        // the generic kernels only: a circuit-specialised kernel may need a
        // run-time compile or a key buffer
        cfg_na = *cfg_in;
        cfg_na.specialize = 1;
        cfg = &cfg_na;
        if (!d_state) return set_error(PBIT_E_INVALID_ARG, "an allocation-free run needs d_state");
        if (cfg->use_graph) return set_error(PBIT_E_INVALID_ARG, "an allocation-free run cannot capture a graph");
    }
    if (!d_hist) return set_error(PBIT_E_INVALID_ARG, "d_hist is NULL");
    if (cfg->init != PBIT_INIT_ZERO && cfg->init != PBIT_INIT_RESUME)
        return set_error(PBIT_E_INVALID_ARG, "bad init mode");
    if (cfg->init == PBIT_INIT_RESUME && !d_state) return set_error(PBIT_E_INVALID_ARG, "RESUME needs d_state");
    if (cfg->hist_mode > 4) return set_error(PBIT_E_INVALID_ARG, "bad hist_mode");
    if (cfg->toggle_mode > 2) return set_error(PBIT_E_INVALID_ARG, "bad toggle_mode");
    if (cfg->persistent > 2) return set_error(PBIT_E_INVALID_ARG, "bad persistent mode");
    if (cfg->wg_per_cu > 16) return set_error(PBIT_E_INVALID_ARG, "wg_per_cu must be <= 16");
    if (cfg->lanes_per_chain != 0 && cfg->lanes_per_chain != 1 && cfg->lanes_per_chain != 2 &&
        cfg->lanes_per_chain != 4 && cfg->lanes_per_chain != 8)
        return set_error(PBIT_E_INVALID_ARG, "lanes_per_chain must be 0, 1, 2, 4 or 8");
    if (cfg->specialize > 2) return set_error(PBIT_E_INVALID_ARG, "bad specialize mode");
    if (cfg->block_size && (cfg->block_size % 64 || cfg->block_size > 256))
        return set_error(PBIT_E_INVALID_ARG, "block_size must be a multiple of 64 in 64..256");
    const uint64_t total = (uint64_t)cfg->burn_in + cfg->sweeps;
    if ((uint64_t)cfg->sweep_offset + total > 0xFFFFFFFFull)
        return set_error(PBIT_E_INVALID_ARG, "sweep counter would wrap");
    if (cfg->use_graph && !stream) return set_error(PBIT_E_INVALID_ARG, "graph replay needs a non-null stream");
    const uint32_t nc = (uint32_t)c->circuits.size();
    if (mh && (mh_circ >= nc || cfg->init != PBIT_INIT_RESUME || cfg->use_graph || total == 0))
        return set_error(PBIT_E_INVALID_ARG, "an MH accept needs a resumed run of some sweeps without a graph");
    for (uint32_t i = 0; i < nc; ++i)
        if (cfg->chains[i] && c->circuits[i].ny && cfg->toggle_mode == 2)
            return set_error(PBIT_E_MODE_UNAVAILABLE,
                             "per-bit cone toggles cannot follow three-qubit products: toggle_mode 2");
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
    pbit_status st = device_blobs(c, &dblob, no_alloc);
    if (st != PBIT_OK) return st;

    // ---- plan (every argument error before any enqueue) --------------------
    std::vector<TuneChoice> choices(nc);
    std::vector<bool> batched(nc, false);
    const std::vector<bool> spec = batch_specialised(c, cfg);
    for (uint32_t i = 0; i < nc; ++i) {
        if (!cfg->chains[i]) continue;
        choices[i] = member_choice(c, i, cfg, total, spec);
        batched[i] = runs_batched(c, i, cfg, spec);
    }
    // circuit-specialised kernels are compiled here, before any enqueue (and
    // outside a graph capture): every kernel the run needs and the handle
    // does not hold yet, on host threads at once, then loaded in order
    compile_jits(c, dev, cfg, choices, batched);
    std::vector<const JitKernel *> jits(nc, nullptr);
    for (uint32_t i = 0; i < nc; ++i) {
        if (!cfg->chains[i] || batched[i] || !choices[i].jit) continue;
        const auto key = std::make_tuple(dev, i, jit_hist_kind(choices[i]));
        auto it = c->jit.find(key);
        if (it != c->jit.end()) {
            jits[i] = &it->second;
        } else if (cfg->specialize == 2) {
            return set_error(PBIT_E_MODE_UNAVAILABLE, "specialised kernel unavailable: " + c->jit_failed[key]);
        } else {
            // the generic kernels serve the run
            pbit_gibbs_cfg g = *cfg;
            g.specialize = 1;
            choices[i] = tune_choice(c, i, cfg->chains[i], total, &g);
        }
    }
    const BatchTuning bt = tune_batch(c, cfg);
    uint64_t group = total;
    if (cfg->sweeps_per_launch) group = std::min<uint64_t>(cfg->sweeps_per_launch, total);
    bool multi_group = group < total;
    for (uint32_t i = 0; i < nc; ++i)
        if (cfg->chains[i] && !batched[i] &&
            (choices[i].group < total || (choices[i].jit && jits[i]->hist_kind == JIT_HIST_KEYS &&
                                          (uint64_t)cfg->chains[i] * cfg->sweeps > KEYS_MAX)))
            multi_group = true;
    uint32_t *state_base = d_state;
    if (!d_state && multi_group) {
        void *p = nullptr;
        st = ensure_buf(c->scratch, dev, std::max<uint64_t>(state_words, 1) * sizeof(uint32_t), &p);
        if (st != PBIT_OK) return st;
        state_base = (uint32_t *)p;
    }

    struct Plan {
        GibbsLaunch a;
        uint32_t Wk;
        bool uniform;
        bool tog;
        bool pair;
        const JitKernel *jit;
        uint32_t lanes_log2;
        uint32_t block;
        size_t lds;
        // bins stored as keys: counted into hist_out afterwards
        uint32_t *hist_out;
        uint64_t keys_n;
        uint32_t bits;
        void *part;      // scratch of the key histogram
        uint32_t circ;
        int lane;        // 0: the caller's stream, k > 0: side stream k - 1
    };
    std::vector<Plan> plans;
    uint64_t keys_words = 0;
    size_t part_bytes = 0;
    // persistent classes
    std::vector<BatchCirc> bcirc;
    std::vector<std::vector<BatchTile>> btiles(3);
    std::vector<std::vector<std::pair<uint64_t, uint32_t>>> border(3);  // (cost, circ) for sorting
    size_t blds[3] = {0, 0, 0};
    std::vector<uint32_t> bcirc_of(nc, 0);
    uint64_t soff = 0;
    for (uint32_t i = 0; i < nc; ++i) {
        const CompiledCircuit &k = c->circuits[i];
        const uint32_t ch = cfg->chains[i];
        if (!ch) continue;
        uint32_t *sp = state_base ? state_base + soff : nullptr;
        soff += (uint64_t)ch * k.W;
        if (batched[i]) {
            const size_t hb = ((size_t)1 << (k.n + k.K)) * 4;
            const bool lh = cfg->hist_mode == 1 || (cfg->hist_mode != 2 && hb <= bt.hist_lds_max);
            const size_t lds = gibbs_lds_bytes(k.blob.data(), true, lh);
            if (lds > LDS_LIMIT) return set_error(PBIT_E_INVALID_ARG, "LDS-privatised histogram does not fit");
            BatchCirc bc;
            bc.blob_off = c->blob_off[i];
            bc.state_off = sp ? (uint64_t)(sp - state_base) : 0;
            bc.hist_off = c->hist_off[i];
            bc.n_chains = ch;
            bc.lds_hist = lh ? 1u : 0u;
            bc.Wk = k.WS;
            bc.pad = 0;
            const int cls = batched_class_of(k.WS);
            bcirc_of[i] = (uint32_t)bcirc.size();
            bcirc.push_back(bc);
            blds[cls] = std::max(blds[cls], lds);
            // cost of one tile: Philox blocks x (Philox + toggle row) per sweep
            const uint64_t cost = (uint64_t)k.blob[H_NBLK] * (40 + ((k.WS + 3) & ~3u)) + 64;
            border[cls].push_back({cost, i});
            continue;
        }
        const TuneChoice &tc = choices[i];
        const size_t lds = tc.jit ? jits[i]->lds_bytes
                                  : (tc.pair ? gibbs_pair_lds_bytes(k.blob.data(), tc.lds_hist)
                                             : gibbs_lds_bytes(k.blob.data(), tc.tog, tc.lds_hist));
        if (lds > LDS_LIMIT) return set_error(PBIT_E_INVALID_ARG, "LDS-privatised histogram does not fit");
        const bool keys = tc.jit && jits[i]->hist_kind == JIT_HIST_KEYS;
        for (uint64_t done = 0, g = 0; done < total; done += g) {
            g = std::min<uint64_t>(tc.group, total - done);
            const uint64_t bin0 = std::max<uint64_t>(done, cfg->burn_in);  // first binned sweep, relative
            if (keys && done + g > bin0) {
                // at most KEYS_MAX keys per launch
                const uint64_t per = std::max<uint64_t>(1, KEYS_MAX / ch);
                if (done + g - bin0 > per) g = bin0 - done + per;
            }
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
            p.a.n_sweeps = (uint32_t)g;
            p.a.bin_from = cfg->sweep_offset + cfg->burn_in;
            p.hist_out = nullptr;
            p.keys_n = 0;
            p.bits = k.n + k.K;
            if (keys) {
                // the kernel indexes keys from its first binned sweep
                p.a.bin_from = (uint32_t)(cfg->sweep_offset + bin0);
                p.hist_out = p.a.hist;
                p.a.hist = nullptr;  // the key buffer, set below
                p.keys_n = done + g > bin0 ? (uint64_t)ch * (done + g - bin0) : 0;
                keys_words = std::max(keys_words, p.keys_n);
                part_bytes = std::max(part_bytes, keyhist_scratch_bytes(p.keys_n, p.bits));
            }
            p.a.resume = done > 0 ? 1u : (cfg->init == PBIT_INIT_RESUME ? 1u : 0u);
            p.a.lds_hist = tc.lds_hist ? 1u : 0u;
            p.Wk = k.WS;
            p.uniform = k.uniform;
            p.tog = tc.tog;
            p.pair = tc.pair;
            p.jit = tc.jit ? jits[i] : nullptr;
            p.lanes_log2 = tc.lanes_log2;
            p.block = tc.jit ? std::min<uint32_t>(tc.block, jits[i]->max_block) : tc.block;
            p.lds = lds;
            p.lane = 0;
            p.part = nullptr;
            p.circ = i;
            plans.push_back(p);
        }
    }
    // Independent circuits run concurrently: each circuit's launches go,
    // whole and in order, to one of the caller's stream and the side
    // streams, the heaviest circuit first to the stream with the least work
    // so far (the persistent launch counts as one circuit), so small launches
    // that leave CUs idle overlap, and key histograms (bound by HBM) overlap
    // sweeps (bound by the VALU).  Each stream has its own key buffer.
    constexpr int LANES = 1 + SIDE_STREAMS;
    int batched_lane = 0;
    bool fork = false;
    {
        std::vector<std::pair<double, uint32_t>> units;  // (work, circuit) of circuits with launches of their own
        std::vector<int> lane_of(nc, 0);
        for (uint32_t i = 0; i < nc; ++i)
            if (cfg->chains[i] && !batched[i]) units.push_back({(double)cfg->chains[i] * (c->circuits[i].h + 1), i});
        fork = units.size() + (bcirc.empty() ? 0 : 1) > 1;
        if (fork) {
            double load[LANES] = {0.0, 0.0, 0.0, 0.0};
            auto pick = [&](double w) {
                int best = 0;
                for (int k = 1; k < LANES; ++k)
                    if (load[k] < load[best]) best = k;
                load[best] += w;
                return best;
            };
            if (!bcirc.empty()) {
                double w = 0.0;
                for (uint32_t i = 0; i < nc; ++i)
                    if (batched[i] && cfg->chains[i]) w += (double)cfg->chains[i] * (c->circuits[i].h + 1);
                batched_lane = pick(w);
            }
            std::stable_sort(units.begin(), units.end(),
                             [](const std::pair<double, uint32_t> &a, const std::pair<double, uint32_t> &b) {
                                 return a.first > b.first;
                             });
            for (const auto &u : units) lane_of[u.second] = pick(u.first);
            for (Plan &p : plans) p.lane = lane_of[p.circ];
        }
    }
    if (no_alloc && (fork || keys_words || !bcirc.empty()))
        return set_error(PBIT_E_INVALID_ARG,
                         "an allocation-free run takes single-circuit launches of the generic kernels");
    SideStreams *side = nullptr;
    if (fork && (st = ensure_side(c->side, dev, &side)) != PBIT_OK) return st;

    // key buffers and partial rows of the key histogram, one of each per
    // stream (the plans of one stream run in order)
    void *d_keys = nullptr, *d_part = nullptr;
    const size_t part_stride = (part_bytes + 255) & ~(size_t)255;
    keys_words = (keys_words + 63) & ~63ull;  // each stream's keys start 256-byte aligned
    if (keys_words) {
        const int nl = fork ? LANES : 1;
        if ((st = ensure_buf(c->keys, dev, keys_words * sizeof(uint32_t) * nl, &d_keys)) != PBIT_OK) return st;
        if ((st = ensure_buf(c->keypart, dev, part_stride * nl, &d_part)) != PBIT_OK) return st;
        for (Plan &p : plans)
            if (p.hist_out) {
                p.a.hist = (uint32_t *)d_keys + keys_words * p.lane;
                p.part = (unsigned char *)d_part + part_stride * p.lane;
            }
    }
    // tiles in decreasing cost order (longest first), 256 chains each
    uint32_t tiles_total = 0;
    for (int cls = 0; cls < 3; ++cls) {
        std::stable_sort(border[cls].begin(), border[cls].end(),
                         [](const std::pair<uint64_t, uint32_t> &a, const std::pair<uint64_t, uint32_t> &b) {
                             return a.first > b.first;
                         });
        for (auto &oc : border[cls]) {
            const uint32_t i = oc.second;
            for (uint32_t c0 = 0; c0 < cfg->chains[i]; c0 += 256) btiles[cls].push_back(BatchTile{bcirc_of[i], c0});
        }
        tiles_total += (uint32_t)btiles[cls].size();
    }
    BatchCirc *d_bcirc = nullptr;
    BatchTile *d_btile[3] = {nullptr, nullptr, nullptr};
    uint32_t *d_queue = nullptr;
    if (!bcirc.empty()) {
        const size_t nb = bcirc.size() * sizeof(BatchCirc);
        const size_t nt = (size_t)tiles_total * sizeof(BatchTile);
        const size_t bytes = nb + nt + 3 * 256 + 256;
        void *p = nullptr;
        if ((st = ensure_buf(c->work, dev, bytes, &p)) != PBIT_OK) return st;
        std::vector<unsigned char> &host = c->work_host[dev];
        std::vector<unsigned char> prev;
        prev.swap(host);
        host.assign(bytes, 0);
        std::memcpy(host.data(), bcirc.data(), nb);
        size_t o = nb;
        for (int cls = 0; cls < 3; ++cls) {
            d_btile[cls] = (BatchTile *)((unsigned char *)p + o);
            std::memcpy(host.data() + o, btiles[cls].data(), btiles[cls].size() * sizeof(BatchTile));
            o += btiles[cls].size() * sizeof(BatchTile);
        }
        o = (o + 255) & ~(size_t)255;
        d_queue = (uint32_t *)((unsigned char *)p + o);
        d_bcirc = (BatchCirc *)p;
        // stream-ordered upload, only when the list changed; the host copy
        // stays alive in the handle until the next change
        if (prev.size() != host.size() || std::memcmp(prev.data(), host.data(), o) != 0 ||
            c->work_uploaded[dev] != p) {
            e = hipMemcpyAsync(p, host.data(), o, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return hip_error(e, "upload of the batched work list");
            c->work_uploaded[dev] = p;
        } else {
            host.swap(prev);
        }
    }
    int cus = 256;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_error(e, "hipDeviceGetAttribute");

    // the MH accept: inside the circuit's first sweep launch when that is the
    // specialised kernel for non-constant magnitudes with one lane per chain
    MhFuse mh_fuse;
    bool mh_fused = false;
    if (mh) {
        for (Plan &p : plans) {
            if (p.circ != mh_circ) continue;
            if (p.jit && p.jit->general && p.lanes_log2 == 0 && p.a.resume && p.a.state && p.a.n_sweeps > 0 &&
                !p.hist_out) {
                mh_fuse.prop = mh->prop;
                mh_fuse.logq_cur = mh->logq_cur;
                mh_fuse.logq_prop = mh->logq_prop;
                mh_fuse.accepts = mh->accepts;
                mh_fuse.step = mh->step;
                p.a.mh = &mh_fuse;
                mh_fused = true;
            }
            break;
        }
    }
    auto lane_stream = [&](int lane) { return lane == 0 ? stream : side->s[lane - 1]; };
    auto enqueue_work = [&]() -> pbit_status {
        for (const Plan &p : plans) {
            const hipStream_t ps = lane_stream(p.lane);
            hipError_t le = p.jit ? jit_launch(*p.jit, p.a, p.lanes_log2, p.block, ps)
                            : p.pair ? launch_gibbs_pair(p.Wk, p.a, p.block, p.lds, ps)
                                     : launch_gibbs(p.Wk, p.uniform, p.tog, p.a, p.block, p.lds, ps);
            if (le != hipSuccess) return hip_error(le, "gibbs kernel launch");
            if (p.hist_out && p.keys_n) {
                le = launch_keyhist(p.a.hist, p.keys_n, p.bits, p.part, p.hist_out, ps);
                if (le != hipSuccess) return hip_error(le, "key histogram launch");
            }
        }
        if (bcirc.empty()) return PBIT_OK;
        const hipStream_t bs = lane_stream(batched_lane);
        for (uint64_t done = 0; done < total; done += group) {
            for (int cls = 0; cls < 3; ++cls) {
                if (btiles[cls].empty()) continue;
                BatchArgs a;
                std::memset(&a, 0, sizeof(a));
                a.circs = d_bcirc;
                a.tiles = d_btile[cls];
                a.ntiles = (uint32_t)btiles[cls].size();
                a.queue = d_queue + cls * 64;
                a.chain_begin = cfg->chain_begin;
                a.seed_lo = (uint32_t)cfg->seed;
                a.seed_hi = (uint32_t)(cfg->seed >> 32);
                a.sweep_begin = (uint32_t)(cfg->sweep_offset + done);
                a.n_sweeps = (uint32_t)std::min<uint64_t>(group, total - done);
                a.bin_from = cfg->sweep_offset + cfg->burn_in;
                a.resume = done > 0 ? 1u : (cfg->init == PBIT_INIT_RESUME ? 1u : 0u);
                uint32_t wg = cfg->wg_per_cu ? cfg->wg_per_cu : bt.wg_per_cu[cls];
                if (blds[cls]) wg = std::min<uint32_t>(wg, std::max<uint32_t>(1, (uint32_t)(LDS_LIMIT / blds[cls])));
                const uint32_t grid = std::min<uint32_t>(a.ntiles, (uint32_t)cus * std::max<uint32_t>(wg, 1));
                hipError_t le = launch_batched(cls, a, dblob, state_base, d_hist, grid, blds[cls], bs);
                if (le != hipSuccess) return hip_error(le, "batched kernel launch");
            }
        }
        return PBIT_OK;
    };
    // fork the side streams from the caller's stream, enqueue, join them back
    // (also after an error, so no side stream is left behind a capture)
    auto enqueue = [&]() -> pbit_status {
        if (mh && !mh_fused) {  // before the fork: every stream's sweeps follow it
            const hipError_t me = launch_mh_accept(c->circuits[mh_circ].WS, *mh, stream);
            if (me != hipSuccess) return hip_error(me, "mh accept");
        }
        if (!fork) return enqueue_work();
        hipError_t fe = hipEventRecord(side->fork, stream);
        for (int k = 0; k < SIDE_STREAMS && fe == hipSuccess; ++k) fe = hipStreamWaitEvent(side->s[k], side->fork, 0);
        if (fe != hipSuccess) return hip_error(fe, "side stream fork");
        const pbit_status ws = enqueue_work();
        for (int k = 0; k < SIDE_STREAMS && fe == hipSuccess; ++k) {
            fe = hipEventRecord(side->join[k], side->s[k]);
            if (fe == hipSuccess) fe = hipStreamWaitEvent(stream, side->join[k], 0);
        }
        if (ws != PBIT_OK) return ws;
        if (fe != hipSuccess) return hip_error(fe, "side stream join");
        return PBIT_OK;
    };

    if (!cfg->use_graph) return enqueue();

    // graph replay keyed by everything that shapes the captured launches
    std::vector<uint64_t> key = {(uint64_t)(uintptr_t)stream, (uint64_t)(uintptr_t)d_state,
                                 (uint64_t)(uintptr_t)d_hist, (uint64_t)(uintptr_t)state_base,
                                 (uint64_t)(uintptr_t)d_bcirc, (uint64_t)(uintptr_t)d_keys,
                                 (uint64_t)(uintptr_t)d_part, cfg->chain_begin, cfg->burn_in, cfg->sweeps,
                                 cfg->seed, cfg->sweep_offset, cfg->init, cfg->sweeps_per_launch, cfg->block_size,
                                 cfg->hist_mode, cfg->toggle_mode, cfg->persistent, cfg->wg_per_cu,
                                 cfg->lanes_per_chain, cfg->specialize, c->tune_epoch};
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

using namespace pbit;

extern "C" pbit_status pbit_launch_shape_get(pbit_circuit c, const pbit_gibbs_cfg *cfg, uint32_t index,
                                             pbit_launch_shape *out) {
    if (!c || !cfg || !cfg->chains || !out) return set_error(PBIT_E_INVALID_ARG, "NULL handle, cfg or out");
    if (index >= c->circuits.size()) return set_error(PBIT_E_INVALID_ARG, "circuit index out of range");
    std::lock_guard<std::mutex> lock(c->mu);
    const CompiledCircuit &k = c->circuits[index];
    const uint64_t total = (uint64_t)cfg->burn_in + cfg->sweeps;
    std::memset(out, 0, sizeof(*out));
    out->kernel_words = k.WS;
    const std::vector<bool> spec = batch_specialised(c, cfg);
    if (runs_batched(c, index, cfg, spec)) {
        const BatchTuning bt = tune_batch(c, cfg);
        const size_t hb = ((size_t)1 << (k.n + k.K)) * 4;
        const bool lh = cfg->hist_mode == 1 || (cfg->hist_mode != 2 && hb <= bt.hist_lds_max);
        out->kernel = PBIT_KERNEL_PERSISTENT;
        out->block = 256;
        out->lds_hist = lh ? 1u : 0u;
        out->toggle_tables = 1;
        out->lds_bytes = (uint32_t)gibbs_lds_bytes(k.blob.data(), true, lh);
        out->sweeps_per_launch = cfg->sweeps_per_launch ? std::min<uint64_t>(cfg->sweeps_per_launch, total) : total;
        return PBIT_OK;
    }
    TuneChoice tc = member_choice(c, index, cfg, total, spec);
    if (tc.jit && cfg->specialize != 2) {
        // a specialisation that failed to build on this device is replaced
        // by the generic kernels
        int dev = 0;
        const uint32_t kind = jit_hist_kind(tc);
        if (!c->jit_failed.empty() && hipGetDevice(&dev) == hipSuccess &&
            c->jit_failed.count(std::make_tuple(dev, index, kind))) {
            pbit_gibbs_cfg g = *cfg;
            g.specialize = 1;
            tc = tune_choice(c, index, cfg->chains[index], total, &g);
        }
    }
    out->kernel = tc.jit ? PBIT_KERNEL_SPECIALISED : (tc.pair ? PBIT_KERNEL_TWO_LANE : PBIT_KERNEL_ONE_LANE);
    out->block = tc.block;
    out->lds_hist = tc.jit ? (jit_hist_kind(tc) & 3u) : (tc.lds_hist ? 1u : 0u);
    out->toggle_tables = tc.tog ? 1u : 0u;
    out->lanes_per_chain = tc.jit ? (1u << tc.lanes_log2) : (tc.pair ? 2u : 1u);
    const size_t hist_lb = tc.lds_hist ? ((size_t)4 << (k.n + k.K)) : 0;
    out->lds_bytes = (uint32_t)(tc.jit && !k.uniform ? jit_general_lds_bytes(k, tc.lds_hist, 256, tc.lanes_log2 != 0)
                                : tc.jit ? jit_rows_bytes(k) + hist_lb + (tc.path_hist ? ((size_t)4 << k.h) : 0)
                                : tc.pair ? gibbs_pair_lds_bytes(k.blob.data(), tc.lds_hist)
                                          : gibbs_lds_bytes(k.blob.data(), tc.tog, tc.lds_hist));
    out->sweeps_per_launch = tc.group;
    return PBIT_OK;
}

extern "C" pbit_status pbit_specialised_source(pbit_circuit c, uint32_t index, uint32_t lds_hist,
                                               uint32_t max_block, char *buf, size_t cap, size_t *len) {
    if (!c || !len) return set_error(PBIT_E_INVALID_ARG, "NULL handle or len");
    if (max_block != 256 && max_block != 512 && max_block != 1024)
        return set_error(PBIT_E_INVALID_ARG, "max_block must be 256, 512 or 1024");
    if (index >= c->circuits.size()) return set_error(PBIT_E_INVALID_ARG, "circuit index out of range");
    const CompiledCircuit &k = c->circuits[index];
    if (lds_hist > 3 && lds_hist != 4 && lds_hist != 5)
        return set_error(PBIT_E_INVALID_ARG, "lds_hist must be 0, 1, 2, 3, 4 or 5");
    if (!k.uniform && (lds_hist & 3u) > 1)
        return set_error(PBIT_E_MODE_UNAVAILABLE, "path counts and keys need every conditional 1/2");
    if (k.uniform && lds_hist > 3)
        return set_error(PBIT_E_MODE_UNAVAILABLE, "the two-wave form is pbit_general_sweep's");
    if (lds_hist == JIT_HIST_PATHS && k.h > 16) return set_error(PBIT_E_TOO_LARGE, "path counts need h <= 16");
    const JitSource src = jit_uniform_source(k, lds_hist, max_block);
    *len = src.text.size() + 1;
    if (buf && cap) {
        const size_t m = std::min(cap - 1, src.text.size());
        std::memcpy(buf, src.text.data(), m);
        buf[m] = '\0';
    }
    return PBIT_OK;
}
