// Library-internal runtime: compiled handle, device images, run planning.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pbit.h"
#include "compile.h"
#include "jit.h"

namespace pbit {

pbit_status set_error(pbit_status st, const std::string &msg);
pbit_status hip_error(hipError_t e, const char *what);

// A device buffer owned by a handle, one per device ordinal.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// Streams beside the caller's on which independent circuits of one run are
// enqueued, forked from and joined back to the caller's stream with events
// (default priority, non-blocking).
constexpr int SIDE_STREAMS = 3;
struct SideStreams {
    hipStream_t s[SIDE_STREAMS] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr;
    hipEvent_t join[SIDE_STREAMS] = {nullptr, nullptr, nullptr};
};

// Autotuned shape of one circuit's single-circuit launches.
struct TunedSingle {
    uint32_t block = 256;
    bool lds_hist = true;
    bool tog = true;
    bool pair = false;
};

// Autotuned persistent-launch shape: workgroups per CU for each width class
// and the largest histogram privatised in LDS.
struct TunedBatch {
    uint32_t wg_per_cu[3] = {4, 3, 2};
    uint32_t hist_lds_max = 16 * 1024;
};

// Captured sweep-group graph, replayed while the run signature is unchanged.
struct GraphCache {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

}  // namespace pbit

struct pbit_circuit_s {
    std::vector<pbit::CompiledCircuit> circuits;
    std::vector<uint64_t> hist_off;
    uint64_t hist_total = 0;
    std::mutex mu;
    std::map<int, pbit::DevBuf> blobs;    // all circuit images, concatenated
    std::vector<uint64_t> blob_off;       // word offset of each circuit's image
    std::map<int, pbit::DevBuf> scratch;  // lattice state between sweep groups
    std::map<int, pbit::DevBuf> work;     // persistent work list (batched runs)
    std::map<int, std::vector<unsigned char>> work_host;  // its host image
    std::map<int, void *> work_uploaded;
    std::map<int, pbit::GraphCache> graphs;
    // autotuned launch shapes (pbit_autotune)
    std::map<uint32_t, pbit::TunedSingle> tuned;
    bool tuned_batch_valid = false;
    pbit::TunedBatch tuned_batch;
    uint64_t tune_epoch = 0;
    // key buffer and partial rows of the key histogram
    std::map<int, pbit::DevBuf> keys;
    std::map<int, pbit::DevBuf> keypart;
    std::map<int, pbit::SideStreams> side;
    // circuit-specialised kernels by (device, circuit, histogram kind JitHist)
    std::map<std::tuple<int, uint32_t, uint32_t>, pbit::JitKernel> jit;
    std::map<std::tuple<int, uint32_t, uint32_t>, std::string> jit_failed;
    std::vector<hipModule_t> jit_groups;  // modules shared by the kernels of one group compile
    ~pbit_circuit_s();
};

namespace pbit {

struct MhArgs;

// With no_alloc the run allocates no device memory and compiles nothing: it
// takes the generic kernels, needs the images resident and d_state, and
// refuses runs that would need library buffers, side streams or a graph.
// With mh (circuit mh_circ, the run resumed from d_state) the run first
// takes that MH accept for every chain: inside the first sweep launch of
// the circuit when it is the circuit-specialised kernel for non-constant
// magnitudes with one lane per chain, else as a launch of its own before
// the sweeps (the same states, counts and accept counters either way).
pbit_status run_gibbs(pbit_circuit c, const pbit_gibbs_cfg *cfg, uint32_t *d_state, uint32_t *d_hist,
                      hipStream_t stream, bool no_alloc = false, const MhArgs *mh = nullptr,
                      uint32_t mh_circ = 0);

// Device image of every circuit of the handle on the current device
// (uploaded on first use; with no_alloc an error if it is not resident).
pbit_status device_blobs(pbit_circuit c, const uint32_t **base, bool no_alloc = false);

}  // namespace pbit
