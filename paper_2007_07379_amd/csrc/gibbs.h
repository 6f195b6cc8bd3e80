// Launch interface of the Gibbs sampling kernel (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pbit {

// Scalar arguments of one launch (passed by value).
struct GibbsArgs {
    uint32_t n_chains;
    uint32_t chain_begin;
    uint32_t seed_lo, seed_hi;
    uint32_t sweep_begin;
    uint32_t n_sweeps;
    uint32_t bin_from;
    uint32_t resume;
    uint32_t lds_hist;
};

// A Metropolis-Hastings accept of independence proposals that a launch takes
// for each chain before its sweeps (the circuit-specialised kernel for
// circuits with non-constant magnitudes, one lane per chain): the same
// arithmetic as mh_accept_kernel, and the post-transition path binned.
struct MhFuse {
    const uint32_t *prop;                  // word-major proposals
    const double *logq_cur, *logq_prop;    // log q of the current paths and of the proposals
    unsigned long long *accepts;           // per-chain accept counters (may be NULL)
    uint32_t step;                         // MH step counter (Philox counter word 0)
};

struct GibbsLaunch {
    const uint32_t *blob;   // device image of the circuit (blob.h)
    uint32_t *state;        // word-major lattice words, n_chains per word; may be NULL
    uint32_t *hist;         // this circuit's uint32[2^(n+K)] histogram
    uint32_t n_chains;
    uint32_t chain_begin;   // global index of local chain 0
    uint32_t seed_lo, seed_hi;
    uint32_t sweep_begin;   // Philox sweep counter of the launch's first sweep
    uint32_t n_sweeps;
    uint32_t bin_from;      // sweeps with counter >= bin_from are binned
    uint32_t resume;        // 1: read the lattice from state; 0: start from all-zero free bits
    uint32_t lds_hist;      // 1: histogram privatised in LDS
    const MhFuse *mh;       // an MH accept before the sweeps (NULL: none; resume must be 1)
};

// LDS bytes a launch needs (toggle tables when `tog`, thresholds, and the
// histogram when privatised).
size_t gibbs_lds_bytes(const uint32_t *host_blob, bool tog, bool lds_hist);

// Launches the kernel compiled for lattice width Wk (one of KERNEL_WIDTHS);
// `tog` selects the LDS toggle-table variant.
hipError_t launch_gibbs(uint32_t Wk, bool uniform, bool tog, const GibbsLaunch &a, uint32_t block,
                        size_t lds_bytes, hipStream_t stream);

// Two-lanes-per-chain variant for circuits whose conditionals are all 1/2
// (gibbs_pair.hip); block is 64..512 threads, i.e. half as many chains.
size_t gibbs_pair_lds_bytes(const uint32_t *host_blob, bool lds_hist);
hipError_t launch_gibbs_pair(uint32_t Wk, const GibbsLaunch &a, uint32_t block, size_t lds_bytes,
                             hipStream_t stream);

}  // namespace pbit
