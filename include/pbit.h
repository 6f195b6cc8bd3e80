/*
 * pbit.h -- C ABI of the MI355X (gfx950) Feynman-path sampler.
 *
 * The problem (Sec. 3 of Chowdhury, Camsari, Datta, "Emulating Quantum
 * Interference with Generalized Ising Machines"): given n qubits, a
 * layered gate sequence U^(1..d) and an input basis state beta, estimate
 * U_{alpha,beta} for every output alpha (Eq. (U)) as the sum over Feynman
 * paths of Eq. (path), by sampling paths with probability proportional to
 * |psi_C| = exp(-Re E) (Eq. (weightedS)) and adding each sample's phase
 * exp(-i Im E) to its output bin (Fig. 2, steps 1-3); Eq. (U23) then turns
 * the bins into amplitudes.
 *
 * Conventions used by every entry point
 *  - Gate matrices are U[out][in] (Sec. 2 one/two-qubit tables).  A
 *    two-qubit gate on (q[0], q[1]) indexes rows and columns by
 *    s_{q[0]} + 2 s_{q[1]} (the column order |00>,|10>,|01>,|11> of
 *    Eq. (ET2)).  Basis states are little-endian: qubit q is bit q.
 *  - The p-bit lattice has d+1 layers of n bits; bit (layer l, qubit q) has
 *    index l*n + q and lives in 32-bit word (l*n+q)/32, bit (l*n+q)%32.
 *    W = ceil(n(d+1)/32) words per chain.
 *  - Zero entries are eliminated exactly (Appendix): a gate whose matrix is
 *    diagonal copies its input p-bits, a gate whose matrix is a permutation
 *    (times phases) fixes its outputs as an affine GF(2) function of its
 *    inputs (NOT, CNOT = XOR), and only gates with no zero entry create new
 *    independent ("free") p-bits.  Other zero patterns are rejected unless
 *    the circuit enables soft zeros (soft_zero_J of pbit_circuit_desc).
 *  - Every nonzero entry must have a phase on the grid 2 pi k / 2^K; the
 *    sample phase is then an integer bin k in [0, 2^K).
 *  - Histograms are uint32[2^n][2^K] (index alpha * 2^K + k), owned and
 *    zeroed by the caller; runs add into them.
 *  - Device buffers are plain device pointers (e.g. a PyTorch tensor's
 *    data_ptr()); streams are hipStream_t passed as void*.  All run entry
 *    points are asynchronous on that stream; results are valid after the
 *    stream is synchronised.
 *  - Errors: negative status codes; argument errors are detected before any
 *    work is enqueued; pbit_last_error() returns a thread-local message.
 *    Device errors surface as PBIT_E_DEVICE.
 *  - Compiled handles are immutable and may be shared by runs on different
 *    streams.
 */
#ifndef PBIT_H
#define PBIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pbit_status;
enum {
    PBIT_OK = 0,
    PBIT_E_INVALID_ARG = -1,
    PBIT_E_UNSUPPORTED_GATE = -2, /* zero pattern neither full, diagonal nor permutation */
    PBIT_E_PHASE_OFF_GRID = -3,   /* an entry's phase is not a multiple of 2 pi / 2^K */
    PBIT_E_TOO_LARGE = -4,        /* lattice > 1024 bits, > 256 free bits, n > 24, ... */
    PBIT_E_DEVICE = -5,
    PBIT_E_COUNT_OVERFLOW = -6,   /* chains x sweeps of one call could overflow a uint32 bin */
    PBIT_E_OOM = -7,
    PBIT_E_MODE_UNAVAILABLE = -8  /* exact-Z normalisation without constant column sums */
};

enum { PBIT_INIT_ZERO = 0, PBIT_INIT_RESUME = 1 };
enum { PBIT_NORM_EXACT_Z = 0, PBIT_NORM_L2 = 1 };

typedef struct pbit_circuit_s *pbit_circuit;
typedef struct pbit_proposal_s *pbit_proposal;

/* One gate.  layer in 1..d; gates of one layer act on disjoint qubits; an
 * idle qubit carries the identity.  re/im hold U[out][in] row-major, the
 * state index s_{q[0]} + 2 s_{q[1]} + 4 s_{q[2]} (2x2 uses the first 4
 * entries, 4x4 the first 16).  One- and two-qubit gates: any zero-free,
 * diagonal or permutation matrix with phases on the 2 pi / 2^K grid.
 * Three-qubit gates: permutation matrices with every nonzero entry 1 (the
 * Appendix's CCNOT and the like: deterministic, their outputs of degree 2
 * in the inputs); a circuit with one whose outputs are not affine needs
 * every other gate's magnitude constant, else UNSUPPORTED_GATE. */
typedef struct {
    uint32_t layer;
    uint32_t arity; /* 1, 2 or 3 */
    uint32_t q[3];
    double re[64];
    double im[64];
} pbit_gate;

/* One circuit.  input_state is beta (bit q = qubit q).  zero_tol: an entry
 * with |U| <= zero_tol is a zero (<= 0 selects 1e-12); phase_tol: allowed
 * distance of arg U from the 2 pi / 2^K grid (<= 0 selects 1e-9).
 * circuit_id (< 2^16) enters every random-number counter. */
typedef struct {
    uint32_t n, d;
    const pbit_gate *gates;
    uint32_t n_gates;
    uint64_t input_state;
    uint32_t K; /* 1..8 */
    double zero_tol, phase_tol;
    uint32_t circuit_id;
    double soft_zero_J; /* 0: a one- or two-qubit gate whose zeros are neither absent nor a
                           permutation pattern is UNSUPPORTED_GATE.  J > 0: soft zeros (Appendix):
                           such a gate samples with e^(-J) in place of its zeros and creates free
                           p-bits; a path that meets one of those entries is not a path of the
                           circuit and is not binned, so the binned law is exact for any J (J only
                           sets how often chains pass through such paths).  Counts then total
                           fewer than chains x sweeps: pass their sum as T to pbit_amplitudes. */
} pbit_circuit_desc;

typedef struct {
    uint32_t n, d, K, W, L; /* L = n (d+1) lattice bits in W words */
    uint32_t h;             /* free p-bits */
    uint32_t n_colours;     /* colours of the free-bit conflict graph */
    uint32_t uniform;       /* 1 if every conditional is exactly 1/2 */
    uint32_t n_gates;
    uint32_t n_quad_offsets; /* distinct index offsets of quadratic phase terms */
    uint32_t hist_bins;      /* 2^(n+K) */
    uint32_t circuit_id;
    int32_t has_exact_z;     /* 1 if Z = product of gate column sums is exact */
    double Z;                /* sum over all paths of |psi_C| (valid if has_exact_z) */
    uint64_t hist_offset;    /* start of this circuit's bins in a set's histogram */
} pbit_circuit_info;

/* Compile n_circuits circuits (Sec. 2 energies Eq. (UE), Appendix
 * eliminations) into one immutable handle ("circuit set").  Host only: no
 * device is needed until the first run.  Returns UNSUPPORTED_GATE,
 * PHASE_OFF_GRID or TOO_LARGE for circuits outside the supported class.
 * The handle is freed with pbit_circuit_free. */
pbit_status pbit_compile_circuit(const pbit_circuit_desc *descs, uint32_t n_circuits,
                                 pbit_circuit *out);
void pbit_circuit_free(pbit_circuit c);
uint32_t pbit_circuit_count(pbit_circuit c);
pbit_status pbit_circuit_info_get(pbit_circuit c, uint32_t idx, pbit_circuit_info *out);

/* Copies the compiled device image of circuit idx (uint32 words) into buf.
 * With buf == NULL only *len (in words) is set.  The layout is documented
 * in paper_2007_07379_amd/csrc/blob.h; it is used to check the compile
 * against an independent one. */
pbit_status pbit_circuit_export(pbit_circuit c, uint32_t idx, uint32_t *buf, size_t *len);

typedef struct {
    const uint32_t *chains;     /* host array: chains per circuit of the set */
    uint32_t chain_begin;       /* global index of each circuit's first chain */
    uint32_t burn_in, sweeps;   /* sweeps not binned, then binned */
    uint64_t seed;              /* Philox key */
    uint32_t sweep_offset;      /* first sweep counter (resume) */
    uint32_t init;              /* PBIT_INIT_ZERO: all free bits 0; RESUME: read d_state */
    uint32_t sweeps_per_launch; /* sweep-group size; 0 = autotuned */
    uint32_t block_size;        /* chains per workgroup (64..256, multiple of 64); 0 = autotuned */
    uint32_t use_graph;         /* 1: replay the sweep groups as a captured hipGraph */
    uint32_t hist_mode;         /* 0 = auto, 1 = LDS-privatised, 2 = global atomics, 3 = path
                                   counts: circuits on the specialised kernel whose 2^h path
                                   table (4 bytes a path) fits in LDS beside the toggle rows count
                                   each sweep's free bits in LDS and bin every path that occurred
                                   once at the end (the same histogram); 4 = keys: circuits on the
                                   specialised kernel with n + K <= 24 and at most 2^24 chains
                                   store each sample's bin
                                   as a 32-bit key (at most 2^28 keys a launch, in a buffer the
                                   handle holds), partitioned by 2^15-bin bucket and counted
                                   through LDS.  Other circuits take 0 for 3 and 4.  Auto
                                   picks 3 for h <= 14 when each path gets >= 16 samples a
                                   workgroup, else LDS bins when they fit, else 4 when HBM
                                   atomics would bound the sweep (few free bits and lattice
                                   words), else 2. */
    uint32_t toggle_mode;       /* 0 = auto, 1 = LDS toggle tables, 2 = per-bit cone toggles
                                   (MODE_UNAVAILABLE for circuits with three-qubit products,
                                   which rebuild the lattice each sweep from the tables) */
    uint32_t persistent;        /* 0 = auto (sets of more than one circuit), 1 = always, 2 = never */
    uint32_t wg_per_cu;         /* persistent grid: workgroups per CU; 0 = autotuned */
    uint32_t lanes_per_chain;   /* 0 = auto, 1, 2, 4 or 8.  Circuits whose conditionals are all
                                   1/2, single-circuit launches only: 2 with the generic kernel
                                   splits a chain's lattice words over two lanes (one lane for
                                   circuits with three-qubit products); with the
                                   specialised kernel L lanes split a chain's sweeps (lane r runs
                                   sweeps r, r + L, ...).  4 and 8 need the specialised kernel.
                                   Other circuits with the specialised kernel: 1 runs one lane
                                   per chain, 2 or more two waves per 64 chains that split each
                                   colour's bits (auto: up to 32,768 chains). */
    uint32_t specialize;        /* 0 = auto (runs of 2^33 updates or more, and any run of a circuit
                                   whose kernel of the needed kind is already compiled in the
                                   handle), 1 = never, 2 = always
                                   (MODE_UNAVAILABLE if the run-time compile fails): a kernel
                                   generated for the circuit and compiled with hipRTC on first use
                                   (cached in the handle); circuits with conditionals other than
                                   1/2 get one lane per chain and the colour schedule unrolled.
                                   In a persistent batch, 2 takes the circuits with at least 512
                                   chains (at most 256, heaviest by chains x free bits first) out
                                   of the batch into launches of their own specialised kernels;
                                   0 does the same when the whole run has 2^33 updates or more,
                                   else takes only members whose own run has that many. */
} pbit_gibbs_cfg;

/* Gibbs sampling of Feynman paths (Fig. 2 steps 1-3): every chain sweeps its
 * free p-bits colour by colour, each update drawing u from Philox4x32-10 at
 * counter (sweep, b/4, chain, circuit_id) (word b%4) and setting the bit to
 * (u < T_b), T_b the uint32 threshold of its exact conditional; after each of
 * the last `sweeps` sweeps the chain adds 1 to hist[alpha * 2^K + k].
 * d_state: device, sum_i chains_i * W_i uint32; circuit i starts at
 *          S_i = sum_{j<i} chains_j * W_j and is word-major (word w of chain
 *          c at S_i + w * chains_i + c); written at the end, read at the
 *          start when init == RESUME; may be NULL with init == ZERO.
 * d_hist:  device, sum_i 2^(n_i+K_i) uint32 at hist_offset; added to.
 * COUNT_OVERFLOW if some chains_i * sweeps >= 2^32.
 * Persistent mode: every circuit with uniform conditionals is cut into
 * tiles of 256 chains, tiles are sorted by decreasing cost and one
 * persistent launch per lattice-width class (W <= 8, <= 17, <= 32) pulls
 * them from an atomic counter; results equal separate runs bit for bit. */
pbit_status pbit_gibbs_run(pbit_circuit c, const pbit_gibbs_cfg *cfg, uint32_t *d_state,
                           uint32_t *d_hist, void *hip_stream);

/* Amplitude recovery (Eqs. (U343), (U23), (U26), (U30); Fig. 2 step 4), host
 * FP64.  counts: host uint64[2^n][2^K] of circuit idx (a run's histogram,
 * possibly summed over runs), T = number of samples.
 * mode EXACT_Z: A_alpha = Z / T sum_k c_{alpha,k} exp(2 pi i k / 2^K) with
 *   sig_re/sig_im the per-component standard deviations of Eq. (U26);
 *   MODE_UNAVAILABLE if the circuit has no exact Z.
 * mode L2: A = B / ||B||_2 with B_alpha = sum_k c_{alpha,k} exp(2 pi i k/2^K);
 *   sig_* are set to zero (the normalisation is itself random).
 * Outputs are host arrays of 2^n doubles (sig_* may be NULL). */
pbit_status pbit_amplitudes(pbit_circuit c, uint32_t idx, const uint64_t *counts, uint64_t T,
                            int mode, double *amp_re, double *amp_im, double *sig_re,
                            double *sig_im);

/* ------------------------------------------------------------------------
 * Learned proposal: a MADE (masked autoregressive MLP) over the n(d+1)
 * lattice positions in lattice order, hidden layers of width `hidden` with
 * ReLU, bf16 weights with FP32 master copies and FP32 accumulation (bf16
 * MFMA), trained on paths the Gibbs chains produce, and used as an
 * independence proposal in Metropolis-Hastings with the exact real energy
 * (Fig. 2 step 2).  Not part of the paper's method (its Boltzmann machine is
 * untrained, Sec. 1); plain Gibbs stays the reference.
 *
 * Parameters, flat FP32, in this order: W1[D][H], b1[H], W2[H][H], b2[H],
 * V[H][D], c[D] (D = n(d+1) positions, H = hidden).  Input position i has
 * degree i+1, hidden unit k degree 1 + floor(k (D-1) / H); a weight from
 * degree a to degree b is kept iff a <= b (output position o has degree o).
 * Masked weights are kept at exactly zero.
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t hidden;    /* width of both hidden layers (multiple of 64); 0 selects 1024 */
    uint64_t seed;      /* initial weights: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from this seed */
} pbit_made_cfg;

typedef struct {
    uint32_t batch;     /* samples per step (<= 16384) */
    uint32_t steps;     /* Adam steps; batches are consecutive, wrapping over the samples */
    float lr, beta1, beta2, eps;  /* 0 selects 1e-3, 0.9, 0.999, 1e-8 */
} pbit_train_cfg;

/* Creates a proposal for circuit idx of c (the handle must outlive it).
 * Errors: PBIT_E_INVALID_ARG for a hidden width that is not a multiple of
 * 64 in 64..4096, PBIT_E_MODE_UNAVAILABLE for circuits with three-qubit
 * products or soft zeros, PBIT_E_TOO_LARGE when no sampler can hold the
 * network's activations in 160 KiB of LDS (made_sample_kernel needs about
 * 32 D + 64 H bytes: H <= 2,304 at D = 400). */
pbit_status pbit_proposal_create(pbit_circuit c, uint32_t idx, const pbit_made_cfg *cfg, pbit_proposal *out);
void pbit_proposal_free(pbit_proposal q);
/* D (positions), H (hidden) and the number of parameters. */
pbit_status pbit_proposal_info(pbit_proposal q, uint32_t *D, uint32_t *H, uint64_t *n_params);
/* Host FP32 parameters in the flat order above; set resets the Adam state
 * and zeroes masked entries. */
pbit_status pbit_proposal_set_params(pbit_proposal q, const float *params, uint64_t n);
pbit_status pbit_proposal_get_params(pbit_proposal q, float *params, uint64_t n);
/* Logits of the given paths (d_states word-major, n paths) into d_logits
 * (device float[n][D]) with the bf16 shadow weights. */
pbit_status pbit_proposal_logits(pbit_proposal q, const uint32_t *d_states, uint32_t n, float *d_logits,
                                 void *hip_stream);
/* Gradient of the batch-mean binary cross-entropy over the free positions
 * (device float[n_params], flat order) and the loss (host, after an
 * internal stream sync). */
pbit_status pbit_proposal_grad(pbit_proposal q, const uint32_t *d_states, uint32_t n, float *d_grad,
                               float *loss_out, void *hip_stream);
/* `steps` Adam steps on batches of d_states (word-major, n_samples paths);
 * losses_out (host, may be NULL) receives one loss per step. */
pbit_status pbit_proposal_train(pbit_proposal q, const uint32_t *d_states, uint64_t n_samples,
                                const pbit_train_cfg *cfg, float *losses_out, void *hip_stream);
/* Draws n independent paths (fused autoregressive sampler; Philox counter
 * (step, b/4, chain_begin + i, circuit_id | 1 << 16), word b%4, for free bit
 * b) into d_out (word-major) with log q of each into d_logq (device double). */
pbit_status pbit_proposal_sample(pbit_proposal q, uint32_t n, uint32_t chain_begin, uint64_t seed,
                                 uint32_t step, uint32_t *d_out, double *d_logq, void *hip_stream);
/* log q of given paths (d_states word-major, valid paths such as chain
 * states or proposals); equal bit for bit to the value the sampler reports
 * for a path it drew.  Networks of width <= 256 are scored by the fused
 * autoregressive kernel with its bits read from d_states, wider ones by the
 * batched forward GEMMs: for widths up to 1,024 on lattices of <= 512 bits
 * with <= 128 free bits (the wide sampler's networks) the logits are then
 * added up in that sampler's order by a replay kernel, for the others by
 * one more GEMM. */
pbit_status pbit_proposal_score(pbit_proposal q, const uint32_t *d_states, uint32_t n, double *d_logq,
                                void *hip_stream);
/* pbit_proposal_sample (n proposals into d_out, d_logq) and
 * pbit_proposal_score of the n word-major paths d_cur (into d_logq_cur) in
 * one call: the MH step's two passes over the network.  For networks of
 * width 64 or 128 whose padded lattice row is 64 or 128 positions (within
 * the register sampler's LDS limit) it is one kernel that carries both
 * paths of a chain through the same weight tiles; otherwise the two calls
 * run in sequence.  Outputs are bit-identical to the two separate calls.
 * d_cur must not overlap d_out. */
pbit_status pbit_proposal_sample_score(pbit_proposal q, uint32_t n, uint32_t chain_begin, uint64_t seed,
                                       uint32_t step, uint32_t *d_out, double *d_logq, const uint32_t *d_cur,
                                       double *d_logq_cur, void *hip_stream);

typedef struct {
    uint32_t chains, chain_begin;
    uint32_t cycles;        /* each cycle: one MH step then gibbs_per_mh Gibbs sweeps */
    uint32_t gibbs_per_mh;  /* 0 allowed */
    uint64_t seed;
    uint32_t step_offset;   /* MH step counter of the first cycle */
    uint32_t sweep_offset;  /* Gibbs sweep counter of the first sweep */
    uint32_t init;          /* PBIT_INIT_ZERO (all free bits 0) or PBIT_INIT_RESUME */
} pbit_mh_cfg;

/* Metropolis-Hastings with the learned independence proposal interleaved
 * with Gibbs sweeps.  Per cycle: propose x' (pbit_proposal_sample), score
 * the current x, accept with probability
 * min(1, |psi(x')| q(x) / (|psi(x)| q(x'))) using Philox word 0 at counter
 * (step, 0, chain, circuit_id | 2 << 16), bin the post-transition path, then
 * gibbs_per_mh Gibbs sweeps each binned.  d_state: word-major W x chains;
 * d_hist as for pbit_gibbs_run; d_accepts: device uint64[chains] (may be
 * NULL), incremented per accepted proposal. */
pbit_status pbit_mh_run(pbit_circuit c, pbit_proposal q, const pbit_mh_cfg *cfg, uint32_t *d_state,
                        uint32_t *d_hist, uint64_t *d_accepts, void *hip_stream);

/* pbit_mh_run for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, and the same states, counts and accept counters bit for
 * bit, but nothing is allocated, freed or compiled: the proposals x' and
 * both log q live in one static device array of 16 MiB per device (held
 * until the process ends), which bounds chains x (4 W + 16) bytes (W =
 * lattice words, each of the three parts rounded up to 256 bytes: about
 * 246,700 chains at W = 13, 699,000 at W = 2; PBIT_E_TOO_LARGE beyond), and the gibbs_per_mh sweeps take the generic
 * (not circuit-specialised) kernels.  Set-up happens in
 * pbit_proposal_create, which places the network, the circuit images and
 * the array's address on the current device; calling on another device is
 * PBIT_E_INVALID_ARG.  Every call on a device shares its array (each call
 * writes all of it that it reads, so nothing carries over), so calls that
 * overlap on one device race: serialise them on one stream. */
pbit_status pbit_mh_run_static(pbit_circuit c, pbit_proposal q, const pbit_mh_cfg *cfg, uint32_t *d_state,
                               uint32_t *d_hist, uint64_t *d_accepts, void *hip_stream);

/* The FP64 natural logarithm whose values the learned proposal's samplers
 * and scorers sum into log q (the log of the threshold probability of each
 * drawn or scored bit), evaluated on n device doubles: d_y[i] = ln(d_x[i])
 * for positive normal d_x[i], within one ulp (x = 2^e m; the top 8 fraction
 * bits of m select a 9-bit inverse G of m's bin, so r = m G - 1 is exact and
 * |r| <= 2^-8; ln x = e ln 2 - ln G + log1p(r), with a table for -ln G split
 * so that its high part and e's share add exactly, and a degree-8 series for
 * log1p).  Exported so its accuracy can be checked against a reference
 * logarithm; device buffers, asynchronous on hip_stream. */
pbit_status pbit_log_eval(const double *d_x, double *d_y, uint64_t n, void *hip_stream);

/* Per-path observables of chain states, for autocorrelation estimates
 * (Eq. (path): a path's output alpha, its phase, the sum of its gates'
 * imaginary energies, and its magnitude exp(-Re E)).  For each of `chains`
 * word-major lattices of circuit idx in d_state (W x chains u32, as
 * pbit_gibbs_run leaves them): d_bin[c] = alpha * 2^K + phi, the histogram
 * bin of the path, and d_logmag[c] = ln|psi_C| up to a constant of the
 * circuit: the FP64 sum of ln|U_g| over the gates whose magnitude is not
 * constant (0 for circuits without such gates).  Device buffers, owned by
 * the caller; either output may be NULL.  Asynchronous on hip_stream. */
pbit_status pbit_path_observables(pbit_circuit c, uint32_t idx, const uint32_t *d_state, uint32_t chains,
                                  uint32_t *d_bin, double *d_logmag, void *hip_stream);

/* Autotuner.  Times candidate launch shapes (workgroup size, lanes per chain, histogram
 * privatisation, toggle tables, sweeps per launch, persistent grid size) on
 * short runs of cfg's workload on hip_stream and keeps the fastest per
 * circuit (and per batched class) in the handle; later runs whose cfg
 * leaves those fields 0 use it.  With cache_path the choices are read from /
 * written to that JSON file, keyed by a hash of the compiled circuits, so a
 * second process skips the timing.  Uses temporary device buffers; blocks
 * until done. */
pbit_status pbit_autotune(pbit_circuit c, const pbit_gibbs_cfg *cfg, const char *cache_path, void *hip_stream);

/* Launch shape that pbit_gibbs_run would use for circuit `index` under
 * cfg (after the handle's autotuned choices and cfg's explicit fields):
 * which kernel, threads per workgroup, histogram privatisation (lds_hist:
 * 0 global atomics, 1 bins in LDS, 2 path counts in LDS, 3 bins stored as
 * keys and counted by a second kernel), toggle tables, the
 * kernel's lattice width in words, LDS bytes and sweeps per launch.  Host
 * only; enqueues nothing. */
enum {
    PBIT_KERNEL_ONE_LANE = 0,   /* one chain per lane */
    PBIT_KERNEL_TWO_LANE = 1,   /* two lanes per chain (all conditionals 1/2) */
    PBIT_KERNEL_PERSISTENT = 2, /* batched persistent tile queue */
    PBIT_KERNEL_SPECIALISED = 3 /* generated for the circuit, compiled at run time */
};
typedef struct {
    uint32_t kernel;
    uint32_t block;
    uint32_t lds_hist;
    uint32_t toggle_tables;
    uint32_t kernel_words;
    uint32_t lds_bytes;
    uint64_t sweeps_per_launch;
    uint32_t lanes_per_chain;
    uint32_t pad;
} pbit_launch_shape;
pbit_status pbit_launch_shape_get(pbit_circuit c, const pbit_gibbs_cfg *cfg, uint32_t index,
                                  pbit_launch_shape *out);

/* HIP source of the specialised sweep kernel of circuit `index`
 * (`pbit_uniform_sweep` when every conditional is 1/2, else
 * `pbit_general_sweep`: the colour schedule unrolled, lds_hist 0 or 1 for
 * one lane per chain, 4 or 5 (= 0 or 1 plus 4) for two waves per 64 chains
 * that split each colour's bits; other values MODE_UNAVAILABLE), with the
 * histogram in global memory (lds_hist 0), its bins privatised in LDS (1),
 * path counts in LDS (2; h <= 16, else TOO_LARGE) or bins stored as keys
 * (3), compiled
 * for workgroups of at most
 * max_block threads (256, 512 or 1024).  Copies at most cap bytes
 * (NUL-terminated) into buf; *len receives the full length + 1.  Host only,
 * for inspection and offline compile checks. */
pbit_status pbit_specialised_source(pbit_circuit c, uint32_t index, uint32_t lds_hist, uint32_t max_block,
                                    char *buf, size_t cap, size_t *len);

/* ------------------------------------------------------------------------
 * Period finding by column sampling (Sec. 5, Figs. 6-7): the first register
 * of the order-finding circuit is n p-bits.  A sample is a configuration x,
 * drawn uniformly (word i mod 4 of Philox4x32-10 at counter (i / 4, 0, 0,
 * 3 << 16) under key seed, its low n bits); f(x) = a^x mod N is the second
 * register; the inverse-QFT column of x, 2^(-n/2) exp(-2 pi i k x / 2^n)
 * over k, is added to column f(x) of psi, and the output law is the row sum
 * of |psi|^2.  With T samples
 *     P[k] = 2^(-n) / T * sum over values f of
 *            |sum over sampled x with f(x) = f of exp(-2 pi i k x / 2^n)|^2,
 * which sums to 1 when no x is drawn twice; its r largest peaks sit near
 * j 2^n / r for the order r of a mod N.
 * ------------------------------------------------------------------------ */
typedef struct {
    uint64_t N;    /* modulus, 3 <= N < 2^31 */
    uint64_t a;    /* base, 1 < a < N (gcd(a, N) = 1 is the caller's concern) */
    uint32_t n;    /* p-bits of the first register, 1 <= n <= 30 */
    uint32_t T;    /* column samples, 1 <= T <= 2^22 */
    uint64_t seed; /* Philox key */
} pbit_shor_cfg;

/* Bytes of device workspace pbit_shor_run needs for cfg (8 x T rounded up
 * to a power of two, at least 32).  Host only. */
pbit_status pbit_shor_work_bytes(const pbit_shor_cfg *cfg, size_t *bytes);

/* Runs the sampler on hip_stream: d_P (caller-owned device buffer of 2^n
 * floats) receives P; d_work (caller-owned device workspace of
 * pbit_shor_work_bytes bytes, 8-byte aligned) holds on return the T samples
 * as uint64 keys (f << 32 | x), sorted by f and then x.  INVALID_ARG for
 * parameters out of range or NULL buffers (before anything is enqueued). */
pbit_status pbit_shor_run(const pbit_shor_cfg *cfg, float *d_P, void *d_work, void *hip_stream);

const char *pbit_last_error(void);

/* Blocks until all work the library enqueued on hip_stream is done; returns
 * PBIT_E_DEVICE if the device reported an error. */
pbit_status pbit_sync(void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* PBIT_H */
