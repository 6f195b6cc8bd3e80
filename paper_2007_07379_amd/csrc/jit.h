// Circuit-specialised sweep kernel for circuits whose conditionals are all
// 1/2 (internal).  The kernel source is generated from one compiled circuit
// and compiled at run time with hipRTC for the current device.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "compile.h"
#include "gibbs.h"

namespace pbit {

// Largest private histogram the specialised kernel keeps in LDS, beside its
// toggle rows.
constexpr size_t JIT_LDS_LIMIT = 160 * 1024;

struct JitSource {
    std::string text;        // HIP source of the kernel `entry`
    std::string entry = "pbit_uniform_sweep";
    uint32_t rows_words = 0; // LDS words of the compacted toggle rows
    uint32_t lds_bytes = 0;  // static LDS of the kernel
    uint32_t xor_words = 0;  // lattice words XORed per sweep (sum of block supports)
    uint32_t max_block = 256;
    bool general = false;     // pbit_general_sweep (takes the MH accept arguments)
};

// Generates the kernel for `k` (k.uniform must hold).  With lds_hist the
// histogram of 2^(n+K) bins is privatised in LDS.  max_block (256, 512 or
// 1024) is the largest workgroup the kernel is compiled for: 1024 threads
// leave 128 VGPRs per lane, 512 leave 256.
// How the generated kernel bins its samples.
enum JitHist : uint32_t {
    JIT_HIST_GLOBAL = 0,  // atomics into the HBM histogram
    JIT_HIST_LDS = 1,     // histogram privatised in LDS, flushed at the end
    // a sweep only draws the free bits and counts the path (bit b = free bit
    // b) in an LDS table of 2^h words (h <= 16); the lattice, phase and bin of
    // every path that occurred are evaluated once per workgroup at the end,
    // so the counts are the same as binning every sample
    JIT_HIST_PATHS = 2,
    // each binned sample's bin is stored as a key: the `hist` argument is then
    // the key buffer, key (s - bin_from) * n_chains + chain for sweep s, with
    // bin_from no earlier than the launch's first sweep (keyhist.h bins them)
    JIT_HIST_KEYS = 3,
    // flag on the kind of pbit_general_sweep: two waves per 64 chains (the
    // bits of Philox block j to wave j & 1, flip flags crossed through LDS
    // once per colour, sweeps of each parity binned by one wave), for runs
    // with too few chains to give each SIMD two waves of one chain a lane
    JIT_PAIRED = 4,
};
// Circuits with other conditionals get the kernel of jit_general_source
// (`pbit_general_sweep`: one lane per chain, LDS or HBM histogram only).
JitSource jit_uniform_source(const CompiledCircuit &k, uint32_t hist_kind, uint32_t max_block);
JitSource jit_general_source(const CompiledCircuit &k, bool lds_hist, uint32_t max_block, bool paired);
// Static LDS of that kernel (threshold tables when they fit, histogram, flip
// masks of the paired form), without generating it.
size_t jit_general_lds_bytes(const CompiledCircuit &k, bool lds_hist, uint32_t max_block, bool paired);

// LDS bytes of the compacted toggle rows (without the histogram).
size_t jit_rows_bytes(const CompiledCircuit &k);

// A compiled, loaded specialisation.
struct JitKernel {
    hipModule_t module = nullptr;  // NULL for a kernel of a shared group module
    hipFunction_t fn = nullptr;
    uint32_t hist_kind = JIT_HIST_GLOBAL;
    uint32_t lds_bytes = 0;
    uint32_t max_block = 256;
    int scratch_bytes = 0;  // per-lane scratch of the compiled kernel (register spills)
    bool general = false;   // pbit_general_sweep: takes the MH accept arguments
};

// Compiles `src` with hipRTC for the current device and loads it (and reads
// back its per-lane scratch size).  On failure returns false and fills `log`.
bool jit_build(const JitSource &src, JitKernel *out, std::string *log);

// The pieces of jit_build.  jit_arch: the current device's target name.
// jit_compile: hipRTC only (no device call); code objects are cached for the
// process by target and source text.  jit_load: loads a code object on the
// current device.
bool jit_arch(std::string *arch, std::string *log);
bool jit_compile(const JitSource &src, const std::string &arch, std::shared_ptr<const std::vector<char>> *code,
                 std::string *log);
bool jit_load(const JitSource &src, const std::vector<char> &code, JitKernel *out, std::string *log);

// Compiles the kernels of srcs as one hipRTC program (each source in a
// namespace of its own, entries renamed) and loads it as one module: hipRTC
// compiles one program at a time per process, and one program of many
// kernels takes about a quarter of the time of as many programs.  On success
// *module is the shared module (the caller unloads it) and out[j] kernel j
// (its own module field NULL).
bool jit_build_group(const std::vector<const JitSource *> &srcs, hipModule_t *module, std::vector<JitKernel> *out,
                     std::string *log);

// Launches a loaded specialisation: lanes_log2 = log2(lanes per chain); lane
// (chain c, residue r) runs the sweeps sweep_begin + r, + r + 2^lanes_log2, ...
// of chain c.  block <= 1024.
hipError_t jit_launch(const JitKernel &k, const GibbsLaunch &a, uint32_t lanes_log2, uint32_t block,
                      hipStream_t stream);

}  // namespace pbit
