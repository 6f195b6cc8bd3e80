// Circuit-specialised sweep kernel for circuits whose conditionals are all
// 1/2, generated from the compiled image and compiled at run time with
// hipRTC.
//
// When every conditional is 1/2 a sweep redraws every free bit from its
// Philox word independently of the lattice, so the lattice after sweep s is
// const ^ XOR_j TOG[j][new bits of block j], whatever came before.  Two
// consequences are used here:
//  * the sweeps of one chain are independent given their counters, so the
//    sweeps of a chain can be split over several lanes (lane r of a chain
//    runs sweeps r, r + L, r + 2L, ...); the lane that runs the chain's last
//    sweep writes its final lattice, and the histogram is a sum over
//    (chain, sweep) either way, so every count and final state equals the
//    one-lane kernel's;
//  * the circuit is fixed for the whole run, so the generated code XORs only
//    the lattice words each block's cones touch (rows compacted to the
//    block's support), evaluates the phase polynomial with its masks as
//    immediates (only nonzero words), and leaves the Philox rounds that the
//    blocks of one sweep share (counter words other than the block index) to
//    common-subexpression elimination.
#include "jit.h"

#include <hip/hiprtc.h>

#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <sstream>

#include "blob.h"

namespace pbit {
namespace {

std::string hx(uint32_t v) {
    char b[16];
    std::snprintf(b, sizeof b, "0x%08xu", v);
    return b;
}

// an exact FP64 literal (hexadecimal significand)
std::string hf(double v) {
    char b[40];
    std::snprintf(b, sizeof b, "(%a)", v);
    return b;
}

std::string xw(uint32_t i, uint32_t W) { return i < W ? "x[" + std::to_string(i) + "]" : std::string("0u"); }

// lattice bits [32 w + delta, 32 w + delta + 32) as one word
std::string funnel(uint32_t w, uint32_t delta, uint32_t W) {
    if (delta < 32)
        return "__builtin_amdgcn_alignbit(" + xw(w + 1, W) + ", " + xw(w, W) + ", " + std::to_string(delta) + "u)";
    return "__builtin_amdgcn_alignbit(" + xw(w + 2, W) + ", " + xw(w + 1, W) + ", " + std::to_string(delta - 32) +
           "u)";
}

// Compacted toggle rows: block j keeps the lattice words its four cones
// touch; row p (p = the four top bits of the block's Philox words) holds the
// XOR of the cones of the bits that come out 1, i.e. the bits whose word has
// its top bit clear (u < 2^31): subset f = p ^ 15.  Blocks start on 16-byte
// boundaries; rows of more than two words are padded to a multiple of four.
struct Blk {
    std::vector<uint32_t> sup;
    uint32_t stride = 1, off = 0;
};

void compact_rows(const CompiledCircuit &k, std::vector<Blk> &blks, std::vector<uint32_t> &rows) {
    const uint32_t *B = k.blob.data();
    const uint32_t W = B[H_W], nblk = B[H_NBLK], TW = B[H_TOGW];
    const uint32_t *tog = B + B[H_OFF_TOG];
    blks.assign(nblk, Blk());
    rows.clear();
    for (uint32_t j = 0; j < nblk; ++j) {
        Blk &b = blks[j];
        for (uint32_t w = 0; w < W; ++w) {
            uint32_t any = 0;
            for (uint32_t f = 0; f < 16; ++f) any |= tog[(j * 16 + f) * TW + w];
            if (any) b.sup.push_back(w);
        }
        const uint32_t s = (uint32_t)b.sup.size();
        b.stride = s <= 2 ? (s ? s : 1) : (s + 3) & ~3u;
        while (rows.size() % 4) rows.push_back(0u);
        b.off = (uint32_t)rows.size();
        for (uint32_t p = 0; p < 16; ++p)
            for (uint32_t i = 0; i < b.stride; ++i)
                rows.push_back(i < s ? tog[(j * 16 + (p ^ 15u)) * TW + b.sup[i]] : 0u);
    }
    while (rows.size() % 4) rows.push_back(0u);
}

const char *PRELUDE = R"(typedef unsigned int u32;
typedef unsigned long long u64;
typedef u32 u32x2 __attribute__((ext_vector_type(2)));
typedef u32 u32x4 __attribute__((ext_vector_type(4)));

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// products, Weyl key schedule.
__device__ __attribute__((always_inline)) inline void philox(u32 c0, u32 c1, u32 c2, u32 c3, u32 k0, u32 k1,
                                       u32 &o0, u32 &o1, u32 &o2, u32 &o3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const u64 p0 = (u64)0xD2511F53u * c0;
        const u64 p1 = (u64)0xCD9E8D57u * c2;
        const u32 n0 = __builtin_amdgcn_bitop3_b32((u32)(p1 >> 32), c1, k0, 0x96);
        const u32 n2 = __builtin_amdgcn_bitop3_b32((u32)(p0 >> 32), c3, k1, 0x96);
        c1 = (u32)p1;
        c3 = (u32)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}
)";

// The phase polynomial and output state of the lattice in x, masks as
// immediates: declares `bin` = alpha 2^K + phase.
void emit_bin_code(std::ostringstream &o, const std::string &ind, const uint32_t *B) {
    const uint32_t W = B[H_W], WS = B[H_WS], K = B[H_K], n = B[H_N];
    for (uint32_t t = 0; t < K; ++t) o << ind << "u32 c" << t << " = 0u;\n";
    const uint32_t linmask = B[H_LINMASK];
    const uint32_t *lin = B + B[H_OFF_LIN];
    for (uint32_t t = 0; t < K; ++t) {
        if (!((linmask >> t) & 1u)) continue;
        for (uint32_t w = 0; w < W; ++w) {
            const uint32_t m = lin[t * WS + w];
            if (m) o << ind << "c" << t << " += __builtin_popcount(x[" << w << "] & " << hx(m) << ");\n";
        }
    }
    const uint32_t *qrec = B + B[H_OFF_QD];
    for (uint32_t q = 0; q < B[H_NQD]; ++q) {
        const uint32_t delta = qrec[0], pm = qrec[1];
        for (uint32_t w = 0; w < W; ++w) {
            bool any = false;
            for (uint32_t t = 0; t < K; ++t)
                if (((pm >> t) & 1u) && qrec[2 + t * WS + w]) any = true;
            if (!any) continue;
            o << ind << "{\n" << ind << "    const u32 y = x[" << w << "] & " << funnel(w, delta, W) << ";\n";
            for (uint32_t t = 0; t < K; ++t) {
                const uint32_t m = qrec[2 + t * WS + w];
                if (((pm >> t) & 1u) && m) o << ind << "    c" << t << " += __builtin_popcount(y & " << hx(m) << ");\n";
            }
            o << ind << "}\n";
        }
        qrec += qd_stride(K, WS);
    }
    const uint32_t *grec = B + B[H_OFF_QG];
    for (uint32_t g = 0; g < B[H_NQG]; ++g) {
        const uint32_t t = grec[0], m = grec[1];
        for (uint32_t w = 0; w < W; ++w) {
            std::string z;
            for (uint32_t e = 0; e < m; ++e) {
                const uint32_t delta = grec[2 + e * qg_entry_stride(WS)];
                const uint32_t mk = grec[2 + e * qg_entry_stride(WS) + 1 + w];
                if (!mk) continue;
                if (!z.empty()) z += " | ";
                z += "(" + funnel(w, delta, W) + " & " + hx(mk) + ")";
            }
            if (!z.empty()) o << ind << "c" << t << " += __builtin_popcount(x[" << w << "] & (" << z << "));\n";
        }
        grec += 2 + m * qg_entry_stride(WS);
    }
    o << ind << "const u32 ph = (" << B[H_PCONST] << "u";
    for (uint32_t t = 0; t < K; ++t) o << " + (c" << t << " << " << t << ")";
    o << ") & " << ((1u << K) - 1u) << "u;\n";
    const uint32_t aw = B[H_AWORD], ash = B[H_ASHIFT];
    o << ind << "const u32 alpha = __builtin_amdgcn_alignbit(" << xw(aw + 1, W) << ", " << xw(aw, W) << ", "
      << ash << "u) & " << hx(n >= 32 ? 0xFFFFFFFFu : (1u << n) - 1u) << ";\n";
    o << ind << "const u32 bin = (alpha << " << K << ") | ph;\n";
}

// True when the lattice in x meets a soft zero (declares `soft_hit`).
void emit_soft_code(std::ostringstream &o, const std::string &ind, const uint32_t *B) {
    const uint32_t ns = B[H_NSOFT];
    const uint32_t *r = B + B[H_OFF_SOFT];
    o << ind << "bool soft_hit = false;\n";
    for (uint32_t g = 0; g < ns; ++g, r += SOFT_STRIDE) {
        o << ind << "soft_hit |= ((" << hx(r[4]) << " >> (";
        for (uint32_t j = 0; j < 4; ++j)
            o << (j ? " | " : "") << "(((x[" << (r[j] >> 5) << "] >> " << (r[j] & 31) << "u) & 1u) << " << j << ")";
        o << ")) & 1u) != 0u;\n";
    }
}

}  // namespace

size_t jit_rows_bytes(const CompiledCircuit &k) {
    std::vector<Blk> blks;
    std::vector<uint32_t> rows;
    compact_rows(k, blks, rows);
    return rows.size() * sizeof(uint32_t);
}

JitSource jit_uniform_source(const CompiledCircuit &k, uint32_t hist_kind, uint32_t max_block) {
    if (!k.uniform)
        return jit_general_source(k, (hist_kind & 3u) == JIT_HIST_LDS, max_block, (hist_kind & JIT_PAIRED) != 0);
    const bool lds_hist = hist_kind == JIT_HIST_LDS, path_hist = hist_kind == JIT_HIST_PATHS;
    const bool keys = hist_kind == JIT_HIST_KEYS;
    const uint32_t *B = k.blob.data();
    const uint32_t W = B[H_W], WS = B[H_WS], K = B[H_K], n = B[H_N], h = B[H_H];
    const uint32_t nblk = B[H_NBLK];
    const uint32_t *cw = B + B[H_OFF_CONST];
    JitSource out;
    out.max_block = max_block;

    std::vector<Blk> blks;
    std::vector<uint32_t> rows;
    compact_rows(k, blks, rows);
    for (const Blk &b : blks) out.xor_words += (uint32_t)b.sup.size();
    out.rows_words = (uint32_t)rows.size();
    const uint32_t nbins = 1u << B[H_HBITS];
    const uint32_t npaths = path_hist ? 1u << h : 0u;
    out.lds_bytes = out.rows_words * 4 + (lds_hist ? nbins * 4 : 0) + npaths * 4;

    // three-qubit permutation gates: each derived AND variable in layer
    // order, read off the lattice so far, its cone XORed in when 1
    auto emit_y = [&](std::ostringstream &o, const std::string &ind) {
        const uint32_t ny = B[H_NY];
        const uint32_t *yr = B + B[H_OFF_Y];
        const uint32_t ys = y_stride(WS);
        for (uint32_t j = 0; j < ny; ++j) {
            const uint32_t p = yr[j * ys], q = yr[j * ys + 1];
            o << ind << "{\n" << ind << "    const u32 m = 0u - ((x[" << (p >> 5) << "] >> " << (p & 31) << "u) & (x["
              << (q >> 5) << "] >> " << (q & 31) << "u) & 1u);\n";
            for (uint32_t w = 0; w < W; ++w) {
                const uint32_t mk = yr[j * ys + 2 + w];
                if (mk) o << ind << "    x[" << w << "] ^= m & " << hx(mk) << ";\n";
            }
            o << ind << "}\n";
        }
    };
    // lattice = const ^ rows of every block, p_j given by an expression
    auto emit_build = [&](std::ostringstream &o, const std::string &ind, auto pexpr) {
        for (uint32_t w = 0; w < W; ++w) o << ind << "x[" << w << "] = " << hx(cw[w]) << ";\n";
        for (uint32_t j = 0; j < nblk; ++j) {
            const Blk &b = blks[j];
            const uint32_t sz = (uint32_t)b.sup.size();
            if (!sz) continue;  // no lattice word depends on this block's bits
            o << ind << "{\n" << ind << "    const u32 p = " << pexpr(j) << ";\n"
              << ind << "    const u32 *r = lds_rows + " << b.off << "u + p * " << b.stride << "u;\n";
            if (b.stride == 1) {
                o << ind << "    x[" << b.sup[0] << "] ^= r[0];\n";
            } else if (b.stride == 2) {
                o << ind << "    const u32x2 v = *(const u32x2 *)r;\n";
                o << ind << "    x[" << b.sup[0] << "] ^= v.x;\n";
                o << ind << "    x[" << b.sup[1] << "] ^= v.y;\n";
            } else {
                for (uint32_t q = 0; q < b.stride / 4; ++q) {
                    o << ind << "    const u32x4 v" << q << " = *(const u32x4 *)(r + " << 4 * q << ");\n";
                    static const char *comp[4] = {"x", "y", "z", "w"};
                    for (uint32_t e = 0; e < 4; ++e) {
                        const uint32_t i = 4 * q + e;
                        if (i < sz) o << ind << "    x[" << b.sup[i] << "] ^= v" << q << "." << comp[e] << ";\n";
                    }
                }
            }
            o << ind << "}\n";
        }
        emit_y(o, ind);
    };
    // phase polynomial and bin of the lattice in x: declares `bin`
    auto emit_bin = [&](std::ostringstream &o, const std::string &ind) { emit_bin_code(o, ind, B); };
    const uint32_t ctag = B[H_CID];  // tag 0: Gibbs updates
    auto from_philox = [&](std::ostringstream &o, const std::string &ind, uint32_t j) {
        o << ind << "u32 u0, u1, u2, u3;\n"
          << ind << "philox(s, " << j << "u, chain, " << hx(ctag) << ", seed_lo, seed_hi, u0, u1, u2, u3);\n";
    };
    auto from_path = [](const std::string &f) {
        return [f](uint32_t j) {
            return "(((" + f + " >> " + std::to_string(4 * j) + ") & 15u) ^ 15u)";
        };
    };

    std::ostringstream o;
    o << PRELUDE;
    o << "\n// circuit: n=" << n << " d=" << B[H_D] << " K=" << K << " W=" << W << " h=" << h
      << " id=" << B[H_CID] << (path_hist ? " (path histogram)" : "") << "\n";
    o << "static __device__ const u32 rows_init[" << out.rows_words << "] = {";
    for (size_t i = 0; i < rows.size(); ++i) o << (i % 8 ? " " : "\n    ") << hx(rows[i]) << ",";
    o << "\n};\n\n";
    o << "extern \"C\" __global__ void __attribute__((amdgpu_flat_work_group_size(1, " << max_block
      << "))) pbit_uniform_sweep(\n"
         "    u32 *__restrict__ state, u32 *__restrict__ hist, u32 n_chains, u32 lanes_log2, u32 chain_begin,\n"
         "    u32 seed_lo, u32 seed_hi, u32 sweep_begin, u32 n_sweeps, u32 bin_from, u32 resume) {\n";
    o << "    __shared__ __attribute__((aligned(16))) u32 lds_rows[" << out.rows_words << "];\n";
    if (lds_hist) o << "    __shared__ u32 lds_h[" << nbins << "];\n";
    if (path_hist) o << "    __shared__ u32 lds_p[" << npaths << "];\n";
    o << "    for (u32 e = threadIdx.x; e < " << out.rows_words << "u; e += blockDim.x) lds_rows[e] = rows_init[e];\n";
    if (lds_hist) o << "    for (u32 e = threadIdx.x; e < " << nbins << "u; e += blockDim.x) lds_h[e] = 0u;\n";
    if (path_hist) o << "    for (u32 e = threadIdx.x; e < " << npaths << "u; e += blockDim.x) lds_p[e] = 0u;\n";
    o << "    __syncthreads();\n";
    o << "    const u32 gl = blockIdx.x * blockDim.x + threadIdx.x;\n"
         "    const u32 lc = gl >> lanes_log2;\n"
         "    const u32 r0 = gl & ((1u << lanes_log2) - 1u);\n"
         "    if (lc < n_chains) {\n"
         "        const u32 chain = chain_begin + lc;\n"
         "        u32 x[" << W << "];\n";
    if (!path_hist) {
        o << "        for (u32 it = r0; it < n_sweeps; it += (1u << lanes_log2)) {\n"
             "            const u32 s = sweep_begin + it;\n";
        // each block's Philox draw, then its row
        for (uint32_t w = 0; w < W; ++w) o << "            x[" << w << "] = " << hx(cw[w]) << ";\n";
        for (uint32_t j = 0; j < nblk; ++j) {
            const Blk &b = blks[j];
            if (b.sup.empty()) continue;
            o << "            {\n";
            from_philox(o, "                ", j);
            o << "                const u32 p = (u0 >> 31) | ((u1 >> 30) & 2u) | ((u2 >> 29) & 4u) | ((u3 >> 28) & 8u);\n"
                 "                const u32 *r = lds_rows + " << b.off << "u + p * " << b.stride << "u;\n";
            const uint32_t sz = (uint32_t)b.sup.size();
            if (b.stride == 1) {
                o << "                x[" << b.sup[0] << "] ^= r[0];\n";
            } else if (b.stride == 2) {
                o << "                const u32x2 v = *(const u32x2 *)r;\n";
                o << "                x[" << b.sup[0] << "] ^= v.x;\n";
                o << "                x[" << b.sup[1] << "] ^= v.y;\n";
            } else {
                for (uint32_t q = 0; q < b.stride / 4; ++q) {
                    o << "                const u32x4 v" << q << " = *(const u32x4 *)(r + " << 4 * q << ");\n";
                    static const char *comp[4] = {"x", "y", "z", "w"};
                    for (uint32_t e = 0; e < 4; ++e) {
                        const uint32_t i = 4 * q + e;
                        if (i < sz) o << "                x[" << b.sup[i] << "] ^= v" << q << "." << comp[e] << ";\n";
                    }
                }
            }
            o << "            }\n";
        }
        emit_y(o, "            ");
        o << "            if (s >= bin_from) {\n";
        emit_bin(o, "                ");
        if (lds_hist)
            o << "                atomicAdd(&lds_h[bin], 1u);\n";
        else if (keys)
            o << "                hist[(u64)(s - bin_from) * n_chains + lc] = bin;\n";
        else
            o << "                atomicAdd(&hist[bin], 1u);\n";
        o << "            }\n";
        o << "        }\n";
    } else {
        // path histogram: a sweep only draws the free bits; the count goes to
        // the path's index (bit b = free bit b), and the lattice, phase and
        // bin of each path that occurred are evaluated once, at the flush
        o << "        u32 last = 0u;\n"
             "        for (u32 it = r0; it < n_sweeps; it += (1u << lanes_log2)) {\n"
             "            const u32 s = sweep_begin + it;\n"
             "            u32 f = 0u;\n";
        for (uint32_t j = 0; j < nblk; ++j) {
            const uint32_t bits = std::min<uint32_t>(4, h - 4 * j);
            o << "            {\n";
            from_philox(o, "                ", j);
            o << "                const u32 p = (u0 >> 31) | ((u1 >> 30) & 2u) | ((u2 >> 29) & 4u) | ((u3 >> 28) & 8u);\n"
                 "                f |= ((p ^ 15u) & " << ((1u << bits) - 1u) << "u) << " << 4 * j << ";\n"
                 "            }\n";
        }
        o << "            if (s >= bin_from) atomicAdd(&lds_p[f], 1u);\n"
             "            last = f;\n"
             "        }\n";
    }
    // final lattice: written by the lane that ran the chain's last sweep
    o << "        if (state && n_sweeps && ((n_sweeps - 1u) & ((1u << lanes_log2) - 1u)) == r0) {\n";
    if (path_hist) emit_build(o, "            ", from_path("last"));
    for (uint32_t w = 0; w < W; ++w)
        o << "            state[(u64)" << w << " * n_chains + lc] = x[" << w << "];\n";
    o << "        }\n";
    o << "    }\n";
    if (lds_hist) {
        o << "    __syncthreads();\n"
             "    for (u32 e = threadIdx.x; e < " << nbins << "u; e += blockDim.x) {\n"
             "        const u32 v = lds_h[e];\n"
             "        if (v) atomicAdd(&hist[e], v);\n"
             "    }\n";
    }
    if (path_hist) {
        o << "    __syncthreads();\n"
             "    for (u32 f = threadIdx.x; f < " << npaths << "u; f += blockDim.x) {\n"
             "        const u32 cnt = lds_p[f];\n"
             "        if (cnt) {\n"
             "            u32 x[" << W << "];\n";
        emit_build(o, "            ", from_path("f"));
        emit_bin(o, "            ");
        o << "            atomicAdd(&hist[bin], cnt);\n"
             "        }\n"
             "    }\n";
    }
    o << "}\n";
    out.text = o.str();
    return out;
}

// Circuits with conditionals other than 1/2: a chain's sweeps depend on each
// other, so lanes cannot split them; the colour schedule is unrolled.  One
// lane per chain, or (paired) two waves per 64 chains that split each
// colour's bits and exchange flip flags through LDS.  Per colour,
// every Philox block the colour needs and no earlier colour drew is drawn
// first (each block once a sweep), then every bit's
// neighbourhood index (its scope bits at immediate positions), threshold
// (from the LDS copy of the tables) and flip are computed, and then the
// flipped bits' cones are XORed in: bits of one colour touch no scope of
// another, so this equals flipping them one after the other.
namespace {

// The free bits of each colour, in the image's colour-entry order.
std::vector<std::vector<uint32_t>> colour_bits(const CompiledCircuit &k) {
    const uint32_t *B = k.blob.data();
    const uint32_t ncol = B[H_NCOL];
    const uint32_t *colidx = B + B[H_OFF_COLIDX];
    const uint32_t *colent = B + B[H_OFF_COLENT];
    std::vector<std::vector<uint32_t>> colbits(ncol);
    for (uint32_t c = 0; c < ncol; ++c)
        for (uint32_t kk = 0; kk < (uint32_t)MAX_FW; ++kk) {
            const uint32_t off = colidx[(c * MAX_FW + kk) * 2], cnt = colidx[(c * MAX_FW + kk) * 2 + 1];
            for (uint32_t e = 0; e < cnt; ++e) {
                const uint32_t blk = colent[off + e] >> 4, msk = colent[off + e] & 15u;
                for (uint32_t t = 0; t < 4; ++t)
                    if ((msk >> t) & 1u) colbits[c].push_back(4 * blk + t);
            }
        }
    return colbits;
}

// Flip-mask words one half of the paired kernel exchanges per colour.
uint32_t flip_mask_words(const std::vector<std::vector<uint32_t>> &colbits) {
    uint32_t fw = 1;
    for (const auto &bits : colbits)
        for (uint32_t hf = 0; hf < 2; ++hf) {
            uint32_t nb = 0;
            for (uint32_t b : bits) nb += ((b >> 2) & 1u) == hf;
            fw = std::max(fw, (nb + 31) / 32);
        }
    return fw;
}

}  // namespace

size_t jit_general_lds_bytes(const CompiledCircuit &k, bool lds_hist, uint32_t max_block, bool paired) {
    const uint32_t *B = k.blob.data();
    const size_t thr = (size_t)B[H_THR_TOTAL] * 4, hist = lds_hist ? ((size_t)4 << B[H_HBITS]) : 0;
    const size_t rows = thr + hist <= JIT_LDS_LIMIT ? thr : 0;
    const size_t flips = paired ? (size_t)2 * max_block * flip_mask_words(colour_bits(k)) * 4 : 0;
    return rows + hist + flips;
}

JitSource jit_general_source(const CompiledCircuit &k, bool lds_hist, uint32_t max_block, bool paired) {
    const uint32_t *B = k.blob.data();
    const uint32_t W = B[H_W], WS = B[H_WS], h = B[H_H], ncol = B[H_NCOL];
    const uint32_t *cw = B + B[H_OFF_CONST];
    const uint32_t *fpos = B + B[H_OFF_FPOS];
    const uint32_t *cone = B + B[H_OFF_CONE];
    const uint32_t *thrinfo = B + B[H_OFF_THRINFO];
    const uint32_t *thrtab = B + B[H_OFF_THRTAB];
    const uint32_t total = B[H_THR_TOTAL];
    const uint32_t nbins = 1u << B[H_HBITS];
    const uint32_t ctag = B[H_CID];
    JitSource out;
    out.entry = "pbit_general_sweep";
    out.general = true;
    out.max_block = max_block;
    const bool thr_lds = (size_t)total * 4 + (lds_hist ? (size_t)nbins * 4 : 0) <= JIT_LDS_LIMIT;
    out.rows_words = thr_lds ? total : 0;

    // the colours' free bits, and (paired) which half handles each: the bits
    // of Philox block j go to half j & 1, so every block is drawn by one half
    const std::vector<std::vector<uint32_t>> colbits = colour_bits(k);
    const uint32_t fw = flip_mask_words(colbits);
    const uint32_t waves = max_block / 64;
    const uint32_t flip_words = paired ? 2 * waves * 64 * fw : 0;
    out.lds_bytes = out.rows_words * 4 + (lds_hist ? nbins * 4 : 0) + flip_words * 4;

    std::ostringstream o;
    o << PRELUDE;
    o << "\n// circuit: n=" << B[H_N] << " d=" << B[H_D] << " K=" << B[H_K] << " W=" << W << " h=" << h
      << " colours=" << ncol << " id=" << B[H_CID] << (paired ? " (two waves per 64 chains)" : "") << "\n";
    o << "static __device__ const u32 thr_init[" << std::max<uint32_t>(total, 1) << "] = {";
    for (uint32_t i = 0; i < std::max<uint32_t>(total, 1); ++i)
        o << (i % 8 ? " " : "\n    ") << hx(i < total ? thrtab[i] : 0u) << ",";
    o << "\n};\n\n";
    // ln|U| tables of the gates with non-constant magnitude (the real-energy
    // records, in gate order) for the MH accept: 4-entry tables become
    // selects, 16-entry ones arrays
    const uint32_t nre = B[H_NRE];
    const uint32_t *re = B + B[H_OFF_RE];
    auto re_val = [&](uint32_t r, uint32_t t) {
        const uint32_t *rec = re + (size_t)r * RE_STRIDE;
        const uint64_t bits = (uint64_t)rec[8 + 2 * t] | ((uint64_t)rec[9 + 2 * t] << 32);
        double v;
        std::memcpy(&v, &bits, sizeof v);
        return v;
    };
    for (uint32_t r = 0; r < nre; ++r) {
        const uint32_t a = re[(size_t)r * RE_STRIDE];
        if (a != 2) continue;
        o << "static __device__ const double mh_re" << r << "[16] = {";
        for (uint32_t t = 0; t < 16; ++t) o << (t % 4 ? " " : "\n    ") << hf(re_val(r, t)) << ",";
        o << "\n};\n";
    }
    o << "extern \"C\" __global__ void __attribute__((amdgpu_flat_work_group_size(1, " << max_block
      << "))) pbit_general_sweep(\n"
         "    u32 *__restrict__ state, u32 *__restrict__ hist, u32 n_chains, u32 lanes_log2, u32 chain_begin,\n"
         "    u32 seed_lo, u32 seed_hi, u32 sweep_begin, u32 n_sweeps, u32 bin_from, u32 resume,\n"
         "    const u32 *__restrict__ mh_prop, const double *__restrict__ mh_lq_cur,\n"
         "    const double *__restrict__ mh_lq_prop, u64 *__restrict__ mh_acc, u32 mh_step) {\n";
    if (thr_lds) o << "    __shared__ u32 lds_t[" << std::max<uint32_t>(total, 1) << "];\n";
    if (lds_hist) o << "    __shared__ u32 lds_h[" << nbins << "];\n";
    if (paired) o << "    __shared__ u32 lds_f[" << flip_words << "];  // [buffer][wave][word][lane]\n";
    if (thr_lds) o << "    for (u32 e = threadIdx.x; e < " << total << "u; e += blockDim.x) lds_t[e] = thr_init[e];\n";
    if (lds_hist) o << "    for (u32 e = threadIdx.x; e < " << nbins << "u; e += blockDim.x) lds_h[e] = 0u;\n";
    o << "    __syncthreads();\n";
    o << "    const u32 *tab = " << (thr_lds ? "lds_t" : "thr_init") << ";\n";
    if (paired) {
        // waves 2g and 2g + 1 of a workgroup run the same 64 chains; every
        // wave runs every sweep (the colours end in workgroup barriers)
        o << "    const u32 wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);\n"
             "    const u32 half = wv & 1u, lane = threadIdx.x & 63u;\n"
             "    const u32 lc = blockIdx.x * (blockDim.x >> 1) + (wv >> 1) * 64u + lane;\n"
             "    const bool valid = lc < n_chains;\n"
             "    {\n";
    } else {
        o << "    const u32 lc = blockIdx.x * blockDim.x + threadIdx.x;\n"
             "    if (lc < n_chains) {\n";
    }
    o << "        const u32 chain = chain_begin + lc;\n"
         "        u32 x[" << W << "];\n"
         "        if (resume" << (paired ? " && valid" : "") << ") {\n";
    for (uint32_t w = 0; w < W; ++w) o << "            x[" << w << "] = state[(u64)" << w << " * n_chains + lc];\n";
    o << "        } else {\n";
    for (uint32_t w = 0; w < W; ++w) o << "            x[" << w << "] = " << hx(cw[w]) << ";\n";
    o << "        }\n";
    if (!paired) {
        // the MH accept of the proposal (one lane per chain only): log r =
        // [ln|psi(y)| - ln|psi(x)|] + [log q(x) - log q(y)], the ln|U| terms
        // added in gate order from zero; accept iff Philox word 0 at
        // (step, 0, chain, id | 2 << 16) < min(1, e^(log r)) 2^32; the
        // post-transition path is binned
        auto bitx = [&](const char *v, uint32_t p) {
            return std::string("((") + v + "[" + std::to_string(p >> 5) + "] >> " + std::to_string(p & 31) + "u) & 1u)";
        };
        o << "        if (mh_prop) {\n"
             "            u32 y[" << W << "];\n";
        for (uint32_t w = 0; w < W; ++w) o << "            y[" << w << "] = mh_prop[(u64)" << w << " * n_chains + lc];\n";
        o << "            double lr = mh_lq_cur[lc] - mh_lq_prop[lc];\n";
        if (nre) {
            o << "            double wx = 0.0, wy = 0.0;\n";
            for (uint32_t r = 0; r < nre; ++r) {
                const uint32_t *rec = re + (size_t)r * RE_STRIDE;
                const uint32_t a = rec[0];
                for (int side = 0; side < 2; ++side) {
                    const char *v = side ? "y" : "x";
                    std::string in = "0u", out = "0u";
                    for (uint32_t j = 0; j < a; ++j) {
                        in += " | (" + bitx(v, rec[1 + j]) + " << " + std::to_string(j) + ")";
                        out += " | (" + bitx(v, rec[3 + j]) + " << " + std::to_string(j) + ")";
                    }
                    const std::string t = std::string("t") + v + std::to_string(r);
                    o << "            const u32 " << t << " = (" << out << ") * " << (1u << a) << "u + (" << in << ");\n";
                    o << "            w" << v << " += ";
                    if (a == 1)
                        o << "(" << t << " & 2u) ? ((" << t << " & 1u) ? " << hf(re_val(r, 3)) << " : " << hf(re_val(r, 2))
                          << ") : ((" << t << " & 1u) ? " << hf(re_val(r, 1)) << " : " << hf(re_val(r, 0)) << ");\n";
                    else
                        o << "mh_re" << r << "[" << t << "];\n";
                }
            }
            o << "            lr += wy - wx;\n";
        }
        o << "            const double acc = lr >= 0.0 ? 1.0 : exp(lr);\n"
             "            u32 m0, m1, m2, m3;\n"
             "            philox(mh_step, 0u, chain, " << hx(ctag | (2u << 16)) << ", seed_lo, seed_hi, m0, m1, m2, m3);\n"
             "            if ((double)m0 < acc * 4294967296.0) {\n";
        for (uint32_t w = 0; w < W; ++w) o << "                x[" << w << "] = y[" << w << "];\n";
        o << "                if (mh_acc) mh_acc[lc] += 1ull;\n"
             "            }\n"
             "            {\n";
        emit_bin_code(o, "                ", B);
        o << (lds_hist ? "                atomicAdd(&lds_h[bin], 1u);\n" : "                atomicAdd(&hist[bin], 1u);\n");
        o << "            }\n"
             "        }\n";
    }
    o << "        for (u32 it = 0; it < n_sweeps; ++it) {\n"
         "            const u32 s = sweep_begin + it;\n";
    if (paired)
        for (uint32_t j = 0; j < (h + 3) / 4; ++j)
            o << "            u32 u" << j << "_0 = 0u, u" << j << "_1 = 0u, u" << j << "_2 = 0u, u" << j << "_3 = 0u;\n";
    // a Philox block serves the free bits 4j..4j+3, which may belong to
    // several colours: it is drawn once per sweep, before the first colour
    // that needs it, and its words stay in registers until the last
    std::vector<bool> drawn((h + 3) / 4, false);
    auto draw = [&](const char *ind, uint32_t j) {
        if (drawn[j]) return;
        drawn[j] = true;
        if (paired)
            o << ind << "philox(s, " << j << "u, chain, " << hx(ctag) << ", seed_lo, seed_hi, u" << j << "_0, u" << j
              << "_1, u" << j << "_2, u" << j << "_3);\n";
        else
            o << ind << "u32 u" << j << "_0, u" << j << "_1, u" << j << "_2, u" << j << "_3;\n"
              << ind << "philox(s, " << j << "u, chain, " << hx(ctag) << ", seed_lo, seed_hi, u" << j << "_0, u" << j
              << "_1, u" << j << "_2, u" << j << "_3);\n";
    };
    // index, threshold and flip flag of free bit b
    auto flip = [&](const char *ind, uint32_t b) {
        const uint32_t *rec = thrinfo + b * THR_STRIDE;
        const uint32_t toff = rec[0], ns = rec[1];
        o << ind << "const u32 i" << b << " = 0u";
        for (uint32_t j = 0; j < ns; ++j)
            o << " | (((x[" << (rec[2 + j] >> 5) << "] >> " << (rec[2 + j] & 31) << "u) & 1u) << " << j << ")";
        o << ";\n";
        const uint32_t p = fpos[b];
        o << ind << "const u32 f" << b << " = (u" << (b >> 2) << "_" << (b & 3) << " < tab[" << toff << "u + i" << b
          << "] ? 1u : 0u) ^ ((x[" << (p >> 5) << "] >> " << (p & 31) << "u) & 1u);\n";
    };
    // XOR of free bit b's cone, under the all-ones-or-zero mask expression m
    auto apply = [&](const char *ind, uint32_t b, const std::string &m) {
        o << ind << "{\n" << ind << "    const u32 m = " << m << ";\n";
        for (uint32_t w = 0; w < W; ++w) {
            const uint32_t mk = cone[(size_t)b * WS + w];
            if (mk) o << ind << "    x[" << w << "] ^= m & " << hx(mk) << ";\n";
        }
        o << ind << "}\n";
    };
    for (uint32_t c = 0; c < ncol; ++c) {
        const std::vector<uint32_t> &bits = colbits[c];
        if (!paired) {
            for (uint32_t b : bits) draw("            ", b >> 2);
            o << "            {  // colour " << c << "\n";
            for (uint32_t b : bits) flip("                ", b);
            for (uint32_t b : bits) apply("                ", b, "0u - f" + std::to_string(b));
            o << "            }\n";
            continue;
        }
        // paired: each half draws its blocks and takes its bits' flips, the
        // flags cross through LDS, and both halves apply every flip
        std::vector<uint32_t> sub[2];
        for (uint32_t b : bits) sub[(b >> 2) & 1u].push_back(b);
        const uint32_t buf = c & 1u;
        o << "            {  // colour " << c << "\n"
             "                u32 mine[" << fw << "] = {";
        for (uint32_t q = 0; q < fw; ++q) o << (q ? ", " : "") << "0u";
        o << "};\n";
        for (uint32_t hf = 0; hf < 2; ++hf) {
            o << "                " << (hf ? "} else {\n" : "if (half == 0u) {\n");
            for (uint32_t b : sub[hf]) draw("                    ", b >> 2);
            for (size_t q = 0; q < sub[hf].size(); ++q) {
                flip("                    ", sub[hf][q]);
                o << "                    mine[" << q / 32 << "] |= f" << sub[hf][q] << " << " << q % 32 << ";\n";
            }
        }
        o << "                }\n";
        for (uint32_t q = 0; q < fw; ++q)
            o << "                lds_f[((" << buf << "u * " << waves << "u + wv) * " << fw << "u + " << q
              << "u) * 64u + lane] = mine[" << q << "];\n";
        o << "                __syncthreads();\n";
        for (uint32_t q = 0; q < fw; ++q)
            o << "                const u32 other" << q << " = lds_f[((" << buf << "u * " << waves << "u + (wv ^ 1u)) * "
              << fw << "u + " << q << "u) * 64u + lane];\n"
              << "                const u32 fa" << q << " = half == 0u ? mine[" << q << "] : other" << q << ";\n"
              << "                const u32 fb" << q << " = half == 0u ? other" << q << " : mine[" << q << "];\n";
        for (uint32_t hf = 0; hf < 2; ++hf)
            for (size_t q = 0; q < sub[hf].size(); ++q)
                apply("                ", sub[hf][q],
                      std::string("0u - ((") + (hf ? "fb" : "fa") + std::to_string(q / 32) + " >> " +
                          std::to_string(q % 32) + ") & 1u)");
        o << "            }\n";
    }
    // the sample of sweep s: every lattice is the same in both halves, which
    // bin the sweeps of their parity
    o << "            if (s >= bin_from" << (paired ? " && (s & 1u) == half && valid" : "") << ") {\n";
    emit_soft_code(o, "                ", B);
    o << "                if (!soft_hit) {\n";
    emit_bin_code(o, "                    ", B);
    if (lds_hist)
        o << "                    atomicAdd(&lds_h[bin], 1u);\n";
    else
        o << "                    atomicAdd(&hist[bin], 1u);\n";
    o << "                }\n"
         "            }\n"
         "        }\n"
         "        if (state && n_sweeps" << (paired ? " && half == 0u && valid" : "") << ") {\n";
    for (uint32_t w = 0; w < W; ++w) o << "            state[(u64)" << w << " * n_chains + lc] = x[" << w << "];\n";
    o << "        }\n"
         "    }\n";
    if (lds_hist)
        o << "    __syncthreads();\n"
             "    for (u32 e = threadIdx.x; e < " << nbins << "u; e += blockDim.x) {\n"
             "        const u32 v = lds_h[e];\n"
             "        if (v) atomicAdd(&hist[e], v);\n"
             "    }\n";
    o << "}\n";
    out.text = o.str();
    return out;
}

namespace {

// Code objects by (target, source): the kernels generated for equal circuit
// images are the same text, so a compile is done once per process whatever
// handle asks for it.
std::mutex g_code_mu;
std::map<std::string, std::shared_ptr<const std::vector<char>>> g_code;

uint64_t fnv1a(const std::string &s, uint64_t h = 1469598103934665603ull) {
    for (unsigned char c : s) h = (h ^ c) * 1099511628211ull;
    return h;
}

}  // namespace

bool jit_arch(std::string *arch, std::string *log) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        *log = "no device";
        return false;
    }
    *arch = prop.gcnArchName;
    return true;
}

bool jit_compile(const JitSource &src, const std::string &arch, std::shared_ptr<const std::vector<char>> *code,
                 std::string *log) {
    // key: the target, the entry and the source text (with its length, so
    // the FNV-1a digest alone never decides equality)
    const std::string key = arch + "|" + src.entry + "|" + std::to_string(src.text.size()) + "|" +
                            std::to_string(fnv1a(src.text));
    {
        std::lock_guard<std::mutex> lock(g_code_mu);
        auto it = g_code.find(key);
        if (it != g_code.end()) {
            *code = it->second;
            return true;
        }
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.text.c_str(), (src.entry + ".hip").c_str(), 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS) {
        *log = "hiprtcCreateProgram failed";
        return false;
    }
    const std::string archopt = std::string("--gpu-architecture=") + arch;
    const char *opts[] = {archopt.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, 7, opts);
    size_t ls = 0;
    if (hiprtcGetProgramLogSize(prog, &ls) != HIPRTC_SUCCESS) ls = 0;
    std::string lg(ls + 1, '\0');
    if (ls && hiprtcGetProgramLog(prog, &lg[0]) != HIPRTC_SUCCESS) lg = "(log unavailable)";
    if (rc != HIPRTC_SUCCESS) {
        *log = "hipRTC compile failed: " + lg;
        (void)hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t cs = 0;
    auto out = std::make_shared<std::vector<char>>();
    bool got = hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs > 0;
    if (got) {
        out->resize(cs);
        got = hiprtcGetCode(prog, out->data()) == HIPRTC_SUCCESS;
    }
    (void)hiprtcDestroyProgram(&prog);
    if (!got) {
        *log = "hipRTC produced no code object";
        return false;
    }
    {
        std::lock_guard<std::mutex> lock(g_code_mu);
        auto it = g_code.emplace(key, out).first;  // a concurrent compile of the same text may have won
        *code = it->second;
    }
    return true;
}

bool jit_load(const JitSource &src, const std::vector<char> &code, JitKernel *out, std::string *log) {
    hipModule_t mod = nullptr;
    hipError_t e = hipModuleLoadData(&mod, code.data());
    if (e != hipSuccess) {
        *log = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
        return false;
    }
    hipFunction_t fn = nullptr;
    e = hipModuleGetFunction(&fn, mod, src.entry.c_str());
    if (e != hipSuccess) {
        (void)hipModuleUnload(mod);
        *log = std::string("hipModuleGetFunction: ") + hipGetErrorString(e);
        return false;
    }
    int scratch = 0;
    e = hipFuncGetAttribute(&scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, fn);
    if (e != hipSuccess) {
        (void)hipModuleUnload(mod);
        *log = std::string("hipFuncGetAttribute: ") + hipGetErrorString(e);
        return false;
    }
    out->module = mod;
    out->fn = fn;
    out->lds_bytes = src.lds_bytes;
    out->max_block = src.max_block;
    out->general = src.general;
    out->scratch_bytes = scratch;
    return true;
}

bool jit_build(const JitSource &src, JitKernel *out, std::string *log) {
    std::string arch;
    std::shared_ptr<const std::vector<char>> code;
    return jit_arch(&arch, log) && jit_compile(src, arch, &code, log) && jit_load(src, *code, out, log);
}

bool jit_build_group(const std::vector<const JitSource *> &srcs, hipModule_t *module, std::vector<JitKernel> *out,
                     std::string *log) {
    *module = nullptr;
    out->assign(srcs.size(), JitKernel());
    if (srcs.empty()) return true;
    std::string arch;
    if (!jit_arch(&arch, log)) return false;
    // kernel j: its source in a namespace of its own (helpers and tables keep
    // their names), its extern "C" entry renamed to <entry>_g<j>
    JitSource all;
    all.entry = "pbit_group";
    std::vector<std::string> names(srcs.size());
    for (size_t j = 0; j < srcs.size(); ++j) {
        std::string text = srcs[j]->text;
        const std::string decl = " " + srcs[j]->entry + "(";
        const size_t at = text.find(decl);
        if (at == std::string::npos || text.find(decl, at + 1) != std::string::npos) {
            *log = "generated source without a unique entry declaration";
            return false;
        }
        names[j] = srcs[j]->entry + "_g" + std::to_string(j);
        text.replace(at, decl.size(), " " + names[j] + "(");
        all.text += "namespace pbit_k" + std::to_string(j) + " {\n" + text + "\n}\n";
    }
    std::shared_ptr<const std::vector<char>> code;
    if (!jit_compile(all, arch, &code, log)) return false;
    hipModule_t mod = nullptr;
    hipError_t e = hipModuleLoadData(&mod, code->data());
    if (e != hipSuccess) {
        *log = std::string("hipModuleLoadData: ") + hipGetErrorString(e);
        return false;
    }
    for (size_t j = 0; j < srcs.size(); ++j) {
        hipFunction_t fn = nullptr;
        int scratch = 0;
        e = hipModuleGetFunction(&fn, mod, names[j].c_str());
        if (e == hipSuccess) e = hipFuncGetAttribute(&scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, fn);
        if (e != hipSuccess) {
            (void)hipModuleUnload(mod);
            out->assign(srcs.size(), JitKernel());
            *log = std::string("kernel of a group: ") + hipGetErrorString(e);
            return false;
        }
        JitKernel &k = (*out)[j];
        k.module = nullptr;  // the group's module, owned by the caller
        k.fn = fn;
        k.lds_bytes = srcs[j]->lds_bytes;
        k.max_block = srcs[j]->max_block;
        k.general = srcs[j]->general;
        k.scratch_bytes = scratch;
    }
    *module = mod;
    return true;
}

hipError_t jit_launch(const JitKernel &k, const GibbsLaunch &a, uint32_t lanes_log2, uint32_t block,
                      hipStream_t stream) {
    const uint64_t lanes = (uint64_t)a.n_chains << lanes_log2;
    if (block == 0 || block > k.max_block || lanes_log2 > 3) return hipErrorInvalidValue;
    const uint64_t grid = (lanes + block - 1) / block;
    if (grid == 0) return hipSuccess;
    // the kernel indexes lanes and sweeps in 32 bits: every lane index and
    // every sweep index plus one stride must fit
    if (grid * block > 0xFFFFFFFFull || a.n_sweeps > 0xFFFFFF00u) return hipErrorInvalidValue;
    uint32_t *state = a.state, *hist = a.hist;
    uint32_t n_chains = a.n_chains, ll = lanes_log2, cb = a.chain_begin, slo = a.seed_lo, shi = a.seed_hi;
    uint32_t sb = a.sweep_begin, ns = a.n_sweeps, bf = a.bin_from, rs = a.resume;
    if (!k.general) {
        if (a.mh) return hipErrorInvalidValue;
        void *args[] = {&state, &hist, &n_chains, &ll, &cb, &slo, &shi, &sb, &ns, &bf, &rs};
        return hipModuleLaunchKernel(k.fn, (uint32_t)grid, 1, 1, block, 1, 1, 0, stream, args, nullptr);
    }
    // the MH accept needs one lane per chain, the chains' states and sweeps
    // after it (its path is written back with the last sweep's)
    if (a.mh && (lanes_log2 != 0 || !a.resume || !state || a.n_sweeps == 0)) return hipErrorInvalidValue;
    const uint32_t *mp = a.mh ? a.mh->prop : nullptr;
    const double *mc = a.mh ? a.mh->logq_cur : nullptr, *mq = a.mh ? a.mh->logq_prop : nullptr;
    unsigned long long *macc = a.mh ? a.mh->accepts : nullptr;
    uint32_t mstep = a.mh ? a.mh->step : 0u;
    void *args[] = {&state, &hist, &n_chains, &ll, &cb, &slo, &shi, &sb, &ns, &bf, &rs, &mp, &mc, &mq, &macc, &mstep};
    return hipModuleLaunchKernel(k.fn, (uint32_t)grid, 1, 1, block, 1, 1, 0, stream, args, nullptr);
}

}  // namespace pbit
