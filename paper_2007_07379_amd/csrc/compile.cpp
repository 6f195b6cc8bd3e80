// Circuit compiler: quantum circuit -> p-bit lattice image for the kernels.
//
// Follows Sec. 2 of the paper (gate energies E = -ln U, Eq. (UE); one- and
// two-qubit tables, Eq. (ET2)) and its Appendix (exact elimination of zero
// entries: diagonal gates reuse their input p-bit, permutation gates fix the
// output as a Boolean function of the input).  Per gate:
//   |U| entries -> magnitudes (exp(-Re E)), arg U -> integer phase bins
//   k with U/|U| = exp(2 pi i k / 2^K) (exp(-i Im E)).
// Lattice: every bit is an affine GF(2) form of the free bits; the cone of
// free bit b is every lattice bit whose form contains b.  A three-qubit
// permutation gate (the Appendix's CCNOT) has outputs of degree 2 in its
// inputs: each product of two input bits becomes a derived variable y
// (the AND of two lattice bits of the previous layer), so every bit is an
// affine form of the free bits and the y's, and the lattice of a sweep is
// the free bits' part followed by the y's in layer order, each y read off
// the lattice so far and its cone XORed in when it is 1.  Such circuits
// must have every conditional 1/2.
// Conditionals (Eq. (weightedS) restricted to one free bit): the factors of
// b are the gates with non-constant magnitude whose scope meets its cone;
// the threshold table over the factors' scope bits holds
//   T = min(floor(w1 / (w0 + w1) * 2^32), 2^32 - 1),
//   w_v = product over factors (ascending gate order) of |U_g| at bit b = v.
// Colouring: free bits whose cones touch each other's factor scopes
// conflict; greedy colouring in ascending free-bit order.
// Soft zeros (Appendix, general zero elements; desc.soft_zero_J > 0): a
// one- or two-qubit gate whose zeros are neither absent nor a permutation
// pattern (controlled Hadamard, controlled rotations) gets e^(-J) in place
// of each zero for sampling and creates free p-bits like a gate without
// zeros; a path that meets one of these entries is not a path of the
// circuit and is not binned, so the binned law is the circuit's exactly.
// The phases at soft entries never reach a binned sample: they are chosen
// (mod 2^K) so that the gate's phase polynomial keeps degree <= 2.
// Phase polynomial: each gate's phase table is expanded as a multilinear
// polynomial over Z_{2^K} in its lattice bits (Moebius transform); the sum
// is stored as bit planes (linear terms per lattice bit, quadratic terms per
// index offset) that the kernel evaluates with popcounts.
//
// Host code; compiled with -ffp-contract=off so FP64 products are exactly
// the IEEE sequence written here.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "blob.h"
#include "compile.h"

namespace pbit {

namespace {

struct Form {
    uint32_t c = 0;
    std::array<uint64_t, MAX_FW / 2> s{};  // 256 free bits
    uint64_t y = 0;                          // derived AND variables
    void xor_with(const Form &o) {
        c ^= o.c;
        for (size_t i = 0; i < s.size(); ++i) s[i] ^= o.s[i];
        y ^= o.y;
    }
    bool has(uint32_t b) const { return (s[b >> 6] >> (b & 63)) & 1u; }
};

struct GateC {
    uint32_t layer, a;
    bool soft[16];  // soft zeros (two-qubit tables at most)
    uint32_t q[3];
    uint32_t in_bits[3], out_bits[3];
    double mag[64];
    int32_t ph[64];  // -1 where the entry is zero
    int kind;        // 0 branching, 1 copy, 2 derived
    uint32_t perm[8];
    bool const_mag;
    bool has_col_sum;
    double col_sum;
};

enum { KIND_BRANCH = 0, KIND_COPY = 1, KIND_DERIVED = 2 };

inline bool getb(const std::vector<uint32_t> &x, uint32_t p) { return (x[p >> 5] >> (p & 31)) & 1u; }
inline void setb(std::vector<uint32_t> &x, uint32_t p) { x[p >> 5] |= 1u << (p & 31); }

pbit_status fail(std::string &err, pbit_status st, const std::string &msg) {
    err = msg;
    return st;
}

// Values at the soft entries of a two-qubit phase table (index o * 4 + i,
// which is also its Moebius index over the bits i0 i1 o0 o1) that make the
// coefficients of degree 3 and 4 vanish mod 2^K: five linear equations
// with coefficients +-1 over Z_(2^K), solved by elimination on odd (unit)
// pivots, free unknowns 0.  False if that finds no solution.
bool complete_soft_phases(int32_t ph[16], const bool soft[16], uint32_t K) {
    const int64_t M = (int64_t)1 << K, MK = M - 1;
    std::vector<uint32_t> unk;
    for (uint32_t t = 0; t < 16; ++t)
        if (soft[t]) unk.push_back(t);
    const uint32_t S_list[5] = {7, 11, 13, 14, 15};
    const size_t nu = unk.size();
    std::vector<std::vector<int64_t>> A(5, std::vector<int64_t>(nu, 0));
    std::vector<int64_t> rhs(5, 0);
    for (int r = 0; r < 5; ++r) {
        const uint32_t S = S_list[r];
        for (uint32_t T = 0; T < 16; ++T) {
            if ((T & S) != T) continue;
            const int64_t sg = (__builtin_popcount(S ^ T) & 1) ? -1 : 1;
            if (soft[T]) {
                for (size_t u = 0; u < nu; ++u)
                    if (unk[u] == T) A[r][u] = (A[r][u] + sg) & MK;
            } else {
                rhs[r] = (rhs[r] - sg * ph[T]) & MK;
            }
        }
    }
    std::vector<int> pivot_col(5, -1);
    std::vector<bool> used(nu, false);
    for (int r = 0; r < 5; ++r) {
        int c = -1;
        for (size_t u = 0; u < nu && c < 0; ++u)
            if (!used[u] && (A[r][u] & 1)) c = (int)u;
        if (c < 0) continue;
        // scale the row by the inverse of its odd pivot (Newton iteration)
        int64_t inv = 1;
        for (int it = 0; it < 6; ++it) inv = (inv * (2 - A[r][c] * inv)) & MK;
        for (size_t u = 0; u < nu; ++u) A[r][u] = (A[r][u] * inv) & MK;
        rhs[r] = (rhs[r] * inv) & MK;
        for (int r2 = 0; r2 < 5; ++r2) {
            if (r2 == r || !A[r2][c]) continue;
            const int64_t f = A[r2][c];
            for (size_t u = 0; u < nu; ++u) A[r2][u] = (A[r2][u] - f * A[r][u]) & MK;
            rhs[r2] = (rhs[r2] - f * rhs[r]) & MK;
        }
        used[c] = true;
        pivot_col[r] = c;
    }
    std::vector<int64_t> val(nu, 0);
    for (int r = 0; r < 5; ++r) {
        if (pivot_col[r] >= 0) {
            val[pivot_col[r]] = rhs[r];
        } else {
            for (size_t u = 0; u < nu; ++u)
                if (A[r][u]) return false;
            if (rhs[r]) return false;
        }
    }
    for (size_t u = 0; u < nu; ++u) ph[unk[u]] = (int32_t)val[u];
    // check: no term of degree 3 or 4 is left
    int64_t f[16];
    for (uint32_t t = 0; t < 16; ++t) f[t] = ph[t];
    for (uint32_t j = 0; j < 4; ++j)
        for (uint32_t a = 0; a < 16; ++a)
            if (a & (1u << j)) f[a] -= f[a ^ (1u << j)];
    for (uint32_t a = 0; a < 16; ++a)
        if (__builtin_popcount(a) >= 3 && (f[a] & MK)) return false;
    return true;
}

}  // namespace

pbit_status compile_one(const pbit_circuit_desc &D, CompiledCircuit &out, std::string &err) {
    const uint32_t n = D.n, d = D.d, K = D.K;
    if (n < 1 || d < 1) return fail(err, PBIT_E_INVALID_ARG, "n and d must be >= 1");
    if (K < 1 || K > (uint32_t)MAX_K) return fail(err, PBIT_E_INVALID_ARG, "K must be in 1..8");
    if (n > (uint32_t)MAX_N || n + K > 28) return fail(err, PBIT_E_TOO_LARGE, "n > 24 or n + K > 28");
    const uint64_t L64 = (uint64_t)n * (d + 1);
    if (L64 > 32u * MAX_W) return fail(err, PBIT_E_TOO_LARGE, "lattice larger than 1024 bits");
    if (D.circuit_id >= (1u << 16)) return fail(err, PBIT_E_INVALID_ARG, "circuit_id >= 2^16");
    if (n < 64 && (D.input_state >> n) != 0) return fail(err, PBIT_E_INVALID_ARG, "input state has bits >= n");
    if (D.n_gates && !D.gates) return fail(err, PBIT_E_INVALID_ARG, "gates is NULL");
    const uint32_t L = (uint32_t)L64;
    const uint32_t W = (L + 31) / 32;
    const uint32_t WS = kernel_words(W);  // stride of per-word arrays in the image
    const double zero_tol = D.zero_tol > 0 ? D.zero_tol : 1e-12;
    const double phase_tol = D.phase_tol > 0 ? D.phase_tol : 1e-9;
    const double step = 2.0 * M_PI / (double)(1u << K);
    const uint32_t KM = (1u << K) - 1;

    // ---- gates: validation, tables, classification ------------------------
    std::vector<GateC> gates(D.n_gates);
    std::vector<int> owner((size_t)(d + 1) * n, -1);
    for (uint32_t gi = 0; gi < D.n_gates; ++gi) {
        const pbit_gate &g = D.gates[gi];
        if (g.arity < 1 || g.arity > 3) return fail(err, PBIT_E_INVALID_ARG, "gate arity must be 1, 2 or 3");
        if (g.layer < 1 || g.layer > d) return fail(err, PBIT_E_INVALID_ARG, "gate layer out of 1..d");
        for (uint32_t j = 0; j < g.arity; ++j)
            if (g.q[j] >= n) return fail(err, PBIT_E_INVALID_ARG, "gate qubit >= n");
        for (uint32_t j = 0; j < g.arity; ++j)
            for (uint32_t t = 0; t < j; ++t)
                if (g.q[j] == g.q[t]) return fail(err, PBIT_E_INVALID_ARG, "gate acts twice on one qubit");
        for (uint32_t j = 0; j < g.arity; ++j) {
            int &o = owner[(size_t)g.layer * n + g.q[j]];
            if (o >= 0) return fail(err, PBIT_E_INVALID_ARG, "gates of one layer overlap");
            o = (int)gi;
        }
        GateC &c = gates[gi];
        c.layer = g.layer;
        c.a = g.arity;
        for (bool &v : c.soft) v = false;
        for (uint32_t j = 0; j < 3; ++j) c.q[j] = j < g.arity ? g.q[j] : 0;
        const uint32_t dim = 1u << c.a;
        bool any_zero = false;
        int row_nz[8] = {0, 0, 0, 0, 0, 0, 0, 0}, col_nz[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (uint32_t o = 0; o < dim; ++o)
            for (uint32_t i = 0; i < dim; ++i) {
                const double re = g.re[o * dim + i], im = g.im[o * dim + i];
                const double m = std::sqrt(re * re + im * im);
                const uint32_t t = o * dim + i;
                if (!(m > zero_tol)) {
                    c.mag[t] = 0.0;
                    c.ph[t] = -1;
                    any_zero = true;
                    continue;
                }
                const double th = std::atan2(im, re);
                const long k = std::lround(th / step);
                if (std::fabs(th - (double)k * step) > phase_tol)
                    return fail(err, PBIT_E_PHASE_OFF_GRID, "gate entry phase is off the 2pi/2^K grid");
                c.mag[t] = m;
                c.ph[t] = (int32_t)(((k % (long)(KM + 1)) + (long)(KM + 1)) & (long)KM);
                row_nz[o]++;
                col_nz[i]++;
            }
        bool mono = true;
        for (uint32_t t = 0; t < dim; ++t) mono = mono && row_nz[t] == 1 && col_nz[t] == 1;
        if (!any_zero) {
            if (c.a == 3) return fail(err, PBIT_E_UNSUPPORTED_GATE, "three-qubit gates must be permutations");
            c.kind = KIND_BRANCH;
        } else if (!mono && D.soft_zero_J > 0.0 && c.a <= 2) {
            // soft zeros: e^(-J) for sampling (below), phases completed
            for (uint32_t t = 0; t < dim * dim; ++t)
                if (c.ph[t] < 0) {
                    c.soft[t] = true;
                    c.ph[t] = 0;
                }
            if (c.a == 2 && !complete_soft_phases(c.ph, c.soft, K))
                return fail(err, PBIT_E_UNSUPPORTED_GATE,
                            "soft-zero gate: no phase polynomial of degree <= 2 fits its nonzero entries");
            c.kind = KIND_BRANCH;
        } else {
            if (!mono) return fail(err, PBIT_E_UNSUPPORTED_GATE,
                                   "gate zero pattern is neither zero-free, diagonal nor a permutation");
            bool ident = true;
            for (uint32_t i = 0; i < dim; ++i) {
                for (uint32_t o = 0; o < dim; ++o)
                    if (c.ph[o * dim + i] >= 0) c.perm[i] = o;
                ident = ident && c.perm[i] == i;
            }
            c.kind = ident ? KIND_COPY : KIND_DERIVED;
            if (c.a == 3)
                for (uint32_t t = 0; t < dim * dim; ++t)
                    if (c.ph[t] > 0 || (c.ph[t] == 0 && std::fabs(c.mag[t] - 1.0) > 1e-9))
                        return fail(err, PBIT_E_UNSUPPORTED_GATE,
                                    "three-qubit permutation gates must have entries exactly 1");
        }
        // column sums of |U| (exact normalisation), soft zeros counted as 0
        double cmx = 0, cmn = 1e300;
        for (uint32_t i = 0; i < dim; ++i) {
            double s = 0;
            for (uint32_t o = 0; o < dim; ++o) s += c.mag[o * dim + i];
            cmx = std::max(cmx, s);
            cmn = std::min(cmn, s);
        }
        c.has_col_sum = (cmx - cmn) <= 1e-9 * cmx;
        c.col_sum = cmx;
        // sampling magnitudes
        for (uint32_t t = 0; t < dim * dim; ++t)
            if (c.soft[t]) c.mag[t] = std::exp(-D.soft_zero_J);
        double mx = 0, mn = 1e300;
        for (uint32_t t = 0; t < dim * dim; ++t)
            if (c.ph[t] >= 0) {
                mx = std::max(mx, c.mag[t]);
                mn = std::min(mn, c.mag[t]);
            }
        c.const_mag = (mx - mn) <= 1e-9 * mx;
        for (uint32_t j = 0; j < c.a; ++j) {
            c.in_bits[j] = (c.layer - 1) * n + c.q[j];
            c.out_bits[j] = c.layer * n + c.q[j];
        }
    }
    // gate order: layer, then lowest qubit
    std::stable_sort(gates.begin(), gates.end(), [](const GateC &x, const GateC &y) {
        uint32_t mx = x.q[0], my = y.q[0];
        for (uint32_t j = 1; j < x.a; ++j) mx = std::min(mx, x.q[j]);
        for (uint32_t j = 1; j < y.a; ++j) my = std::min(my, y.q[j]);
        return x.layer != y.layer ? x.layer < y.layer : mx < my;
    });
    const uint32_t G = (uint32_t)gates.size();

    // ---- affine forms over the free bits and the derived AND variables -----
    std::vector<Form> form(L);
    std::vector<std::array<uint32_t, 2>> yvar;  // lattice bits whose AND each y is
    for (uint32_t q = 0; q < n; ++q) form[q].c = (uint32_t)((D.input_state >> q) & 1u);
    std::vector<uint32_t> fpos;
    {
        std::vector<int> at((size_t)(d + 1) * n, -1);  // gate index per (layer, qubit)
        for (uint32_t gi = 0; gi < G; ++gi)
            for (uint32_t j = 0; j < gates[gi].a; ++j) at[(size_t)gates[gi].layer * n + gates[gi].q[j]] = (int)gi;
        for (uint32_t l = 1; l <= d; ++l) {
            for (uint32_t q = 0; q < n; ++q) {
                const int gi = at[(size_t)l * n + q];
                const uint32_t p = l * n + q;
                if (gi < 0) {
                    form[p] = form[p - n];
                } else if (gates[gi].kind == KIND_BRANCH) {
                    if (fpos.size() >= 32u * MAX_FW) return fail(err, PBIT_E_TOO_LARGE, "more than 256 free p-bits");
                    const uint32_t b = (uint32_t)fpos.size();
                    fpos.push_back(p);
                    form[p] = Form();
                    form[p].s[b >> 6] |= 1ull << (b & 63);
                }
            }
            for (uint32_t gi = 0; gi < G; ++gi) {
                const GateC &g = gates[gi];
                if (g.layer != l || g.kind == KIND_BRANCH) continue;
                // out_j as a polynomial over GF(2) in the inputs (Moebius
                // transform of its truth table): every permutation of <= 2
                // bits is affine; of 3 bits, each output is balanced, so of
                // degree <= 2, and a product in_t in_u becomes a y variable
                const uint32_t dim = 1u << g.a;
                Form nf[3];
                uint32_t ypair[3][3];
                for (auto &r : ypair)
                    for (auto &v : r) v = ~0u;
                for (uint32_t j = 0; j < g.a; ++j) {
                    uint32_t anf[8];
                    for (uint32_t i = 0; i < dim; ++i) anf[i] = (g.perm[i] >> j) & 1u;
                    for (uint32_t t = 0; t < g.a; ++t)
                        for (uint32_t i = 0; i < dim; ++i)
                            if (i & (1u << t)) anf[i] ^= anf[i ^ (1u << t)];
                    nf[j] = Form();
                    nf[j].c = anf[0];
                    for (uint32_t m = 1; m < dim; ++m) {
                        if (!anf[m]) continue;
                        const int deg = __builtin_popcount(m);
                        if (deg == 1) {
                            nf[j].xor_with(form[g.in_bits[__builtin_ctz(m)]]);
                        } else if (deg == 2) {
                            const uint32_t t = __builtin_ctz(m), u = 31 - __builtin_clz(m);
                            if (ypair[t][u] == ~0u) {
                                if (yvar.size() >= 64)
                                    return fail(err, PBIT_E_TOO_LARGE, "more than 64 products in permutation gates");
                                ypair[t][u] = (uint32_t)yvar.size();
                                yvar.push_back({g.in_bits[t], g.in_bits[u]});
                            }
                            nf[j].y ^= 1ull << ypair[t][u];
                        } else {
                            return fail(err, PBIT_E_UNSUPPORTED_GATE, "permutation gate output of degree 3");
                        }
                    }
                }
                for (uint32_t j = 0; j < g.a; ++j) form[g.out_bits[j]] = nf[j];
            }
        }
    }
    const uint32_t h = (uint32_t)fpos.size();
    const uint32_t FW = (h + 31) / 32;

    // cones
    std::vector<std::vector<uint32_t>> cone(h, std::vector<uint32_t>(W, 0));
    for (uint32_t p = 0; p < L; ++p)
        for (uint32_t b = 0; b < h; ++b)
            if (form[p].has(b)) cone[b][p >> 5] |= 1u << (p & 31);
    std::vector<uint32_t> constw(W, 0);
    for (uint32_t p = 0; p < L; ++p)
        if (form[p].c) constw[p >> 5] |= 1u << (p & 31);
    const uint32_t ny = (uint32_t)yvar.size();
    std::vector<std::vector<uint32_t>> ycone(ny, std::vector<uint32_t>(W, 0));
    for (uint32_t p = 0; p < L; ++p)
        for (uint32_t j = 0; j < ny; ++j)
            if ((form[p].y >> j) & 1u) ycone[j][p >> 5] |= 1u << (p & 31);

    // ---- factors, threshold tables, colouring -----------------------------
    auto gate_scope_meets = [&](const GateC &g, const std::vector<uint32_t> &mask) {
        for (uint32_t j = 0; j < g.a; ++j)
            if (getb(mask, g.in_bits[j]) || getb(mask, g.out_bits[j])) return true;
        return false;
    };
    std::vector<std::vector<uint32_t>> factors(h);
    std::vector<std::vector<uint32_t>> fscope(h, std::vector<uint32_t>(W, 0));
    bool uniform = true;
    for (uint32_t b = 0; b < h; ++b) {
        for (uint32_t gi = 0; gi < G; ++gi) {
            if (gates[gi].const_mag) continue;
            if (gate_scope_meets(gates[gi], cone[b])) {
                factors[b].push_back(gi);
                for (uint32_t j = 0; j < gates[gi].a; ++j) {
                    setb(fscope[b], gates[gi].in_bits[j]);
                    setb(fscope[b], gates[gi].out_bits[j]);
                }
            }
        }
        if (!factors[b].empty()) uniform = false;
    }
    if (ny && !uniform)
        return fail(err, PBIT_E_UNSUPPORTED_GATE,
                    "three-qubit gates with products need every gate magnitude constant (all conditionals 1/2)");
    std::vector<uint32_t> colour(h, 0);
    uint32_t ncol = h ? 1 : 0;
    for (uint32_t b = 0; b < h; ++b) {
        std::vector<bool> used(h + 1, false);
        for (uint32_t b2 = 0; b2 < b; ++b2) {
            bool conflict = false;
            for (uint32_t w = 0; w < W && !conflict; ++w)
                conflict = (cone[b2][w] & fscope[b][w]) || (cone[b][w] & fscope[b2][w]);
            if (conflict) used[colour[b2]] = true;
        }
        uint32_t c = 0;
        while (used[c]) ++c;
        colour[b] = c;
        ncol = std::max(ncol, c + 1);
    }

    // threshold tables over S'_b = scope(F_b) + {pos_b}
    std::vector<uint32_t> thrinfo((size_t)h * THR_STRIDE, 0);
    std::vector<uint32_t> thrtab;
    if (!uniform) {
        for (uint32_t b = 0; b < h; ++b) {
            std::vector<uint32_t> S;
            std::vector<uint32_t> sc = fscope[b];
            setb(sc, fpos[b]);
            for (uint32_t p = 0; p < L; ++p)
                if (getb(sc, p)) S.push_back(p);
            if (S.size() > (size_t)MAX_SCOPE)
                return fail(err, PBIT_E_TOO_LARGE, "a conditional depends on more than 12 lattice bits");
            uint32_t *rec = &thrinfo[(size_t)b * THR_STRIDE];
            rec[0] = (uint32_t)thrtab.size();
            rec[1] = (uint32_t)S.size();
            for (size_t j = 0; j < S.size(); ++j) rec[2 + j] = S[j];
            const uint32_t ns = (uint32_t)S.size();
            int jb = -1;
            for (uint32_t j = 0; j < ns; ++j)
                if (S[j] == fpos[b]) jb = (int)j;
            std::vector<uint32_t> x(W, 0);
            for (uint32_t idx = 0; idx < (1u << ns); ++idx) {
                const uint32_t cur = (idx >> jb) & 1u;
                double w[2];
                for (uint32_t v = 0; v < 2; ++v) {
                    std::fill(x.begin(), x.end(), 0u);
                    for (uint32_t j = 0; j < ns; ++j) {
                        uint32_t bit = (idx >> j) & 1u;
                        if (cur != v && getb(cone[b], S[j])) bit ^= 1u;
                        if (bit) setb(x, S[j]);
                    }
                    double pr = 1.0;
                    for (uint32_t gi : factors[b]) {
                        const GateC &g = gates[gi];
                        uint32_t ii = 0, oo = 0;
                        for (uint32_t j = 0; j < g.a; ++j) {
                            ii |= (uint32_t)getb(x, g.in_bits[j]) << j;
                            oo |= (uint32_t)getb(x, g.out_bits[j]) << j;
                        }
                        pr = pr * g.mag[oo * (1u << g.a) + ii];
                    }
                    w[v] = pr;
                }
                double P = w[1] / (w[0] + w[1]);
                double t = std::floor(P * 4294967296.0);
                if (!(t <= 4294967295.0)) t = 4294967295.0;  // also maps NaN (0/0) to the top
                thrtab.push_back((uint32_t)t);
            }
        }
    }

    // ---- phase polynomial ---------------------------------------------------
    uint32_t pconst = 0;
    std::vector<uint32_t> lin(L, 0);
    std::map<std::pair<uint32_t, uint32_t>, uint32_t> quad;
    for (uint32_t gi = 0; gi < G; ++gi) {
        const GateC &g = gates[gi];
        const uint32_t dim = 1u << g.a;
        // variables: inputs, then (branching gates only) outputs
        std::vector<uint32_t> var;
        for (uint32_t j = 0; j < g.a; ++j) var.push_back(g.in_bits[j]);
        if (g.kind == KIND_BRANCH)
            for (uint32_t j = 0; j < g.a; ++j) var.push_back(g.out_bits[j]);
        const uint32_t nv = (uint32_t)var.size();
        std::vector<int64_t> f(1u << nv);
        for (uint32_t a = 0; a < (1u << nv); ++a) {
            uint32_t i = a & (dim - 1);
            uint32_t o = g.kind == KIND_BRANCH ? (a >> g.a) : g.perm[i];
            f[a] = g.ph[o * dim + i];
        }
        // Moebius transform: coefficient of the monomial prod_{j in S} var_j
        for (uint32_t j = 0; j < nv; ++j)
            for (uint32_t a = 0; a < (1u << nv); ++a)
                if (a & (1u << j)) f[a] -= f[a ^ (1u << j)];
        for (uint32_t a = 0; a < (1u << nv); ++a) {
            const uint32_t c = (uint32_t)(((f[a] % (int64_t)(KM + 1)) + (int64_t)(KM + 1)) & (int64_t)KM);
            if (!c) continue;
            const int deg = __builtin_popcount(a);
            if (deg == 0) {
                pconst = (pconst + c) & KM;
            } else if (deg == 1) {
                const uint32_t p = var[__builtin_ctz(a)];
                lin[p] = (lin[p] + c) & KM;
            } else if (deg == 2) {
                uint32_t p0 = var[__builtin_ctz(a)];
                uint32_t p1 = var[31 - __builtin_clz(a)];
                if (p0 > p1) std::swap(p0, p1);
                if (p0 == p1) {
                    lin[p0] = (lin[p0] + c) & KM;
                } else {
                    uint32_t &e = quad[{p1 - p0, p0}];
                    e = (e + c) & KM;
                }
            } else {
                return fail(err, PBIT_E_UNSUPPORTED_GATE, "gate phase polynomial has degree > 2");
            }
        }
    }
    std::vector<uint32_t> linp((size_t)K * WS, 0);
    uint32_t linmask = 0;
    for (uint32_t p = 0; p < L; ++p)
        for (uint32_t t = 0; t < K; ++t)
            if ((lin[p] >> t) & 1u) {
                linp[(size_t)t * WS + (p >> 5)] |= 1u << (p & 31);
                linmask |= 1u << t;
            }
    std::map<uint32_t, std::vector<uint32_t>> qd;  // delta -> planes
    for (auto &kv : quad) {
        if (!kv.second) continue;
        const uint32_t delta = kv.first.first, p0 = kv.first.second;
        if (delta >= 64) return fail(err, PBIT_E_TOO_LARGE, "quadratic phase term spans >= 64 lattice bits");
        auto &pl = qd[delta];
        if (pl.empty()) pl.assign((size_t)K * WS, 0);
        for (uint32_t t = 0; t < K; ++t)
            if ((kv.second >> t) & 1u) pl[(size_t)t * WS + (p0 >> 5)] |= 1u << (p0 & 31);
    }
    if (qd.size() > (size_t)MAX_QD) return fail(err, PBIT_E_TOO_LARGE, "too many quadratic phase offsets");

    // ---- colour schedule: per colour, per free-bit word, Philox blocks ------
    std::vector<uint32_t> colidx((size_t)ncol * MAX_FW * 2, 0);
    std::vector<uint32_t> colent;
    for (uint32_t c = 0; c < ncol; ++c)
        for (uint32_t k = 0; k < (uint32_t)MAX_FW; ++k) {
            colidx[((size_t)c * MAX_FW + k) * 2] = (uint32_t)colent.size();
            for (uint32_t j = 8 * k; j < 8 * k + 8 && 4 * j < h; ++j) {
                uint32_t m = 0;
                for (uint32_t t = 0; t < 4; ++t)
                    if (4 * j + t < h && colour[4 * j + t] == c) m |= 1u << t;
                if (m) colent.push_back((j << 4) | m);
            }
            colidx[((size_t)c * MAX_FW + k) * 2 + 1] = (uint32_t)colent.size() - colidx[((size_t)c * MAX_FW + k) * 2];
        }

    // ---- assemble the blob ----------------------------------------------------
    std::vector<uint32_t> blob(H_COUNT, 0);
    auto append = [&](const std::vector<uint32_t> &v) {
        uint32_t off = (uint32_t)blob.size();
        blob.insert(blob.end(), v.begin(), v.end());
        return off;
    };
    blob[H_MAGIC] = BLOB_MAGIC;
    blob[H_N] = n;
    blob[H_D] = d;
    blob[H_K] = K;
    blob[H_W] = W;
    blob[H_H] = h;
    blob[H_L] = L;
    blob[H_CID] = D.circuit_id;
    blob[H_NCOL] = ncol;
    blob[H_UNIFORM] = uniform ? 1u : 0u;
    blob[H_AWORD] = (d * n) >> 5;
    blob[H_ASHIFT] = (d * n) & 31;
    blob[H_PCONST] = pconst;
    blob[H_LINMASK] = linmask;
    blob[H_FW] = FW;
    blob[H_WS] = WS;
    constw.resize(WS, 0u);
    blob[H_OFF_CONST] = append(constw);
    blob[H_OFF_FPOS] = append(fpos);
    {
        std::vector<uint32_t> flat;
        for (uint32_t b = 0; b < h; ++b) {
            flat.insert(flat.end(), cone[b].begin(), cone[b].end());
            flat.resize((size_t)(b + 1) * WS, 0u);
        }
        blob[H_OFF_CONE] = append(flat);
    }
    blob[H_OFF_LIN] = append(linp);
    {
        // Offsets whose terms sit in one bit plane are merged into groups of
        // pairwise disjoint masks (greedy, ascending delta); offsets with
        // several planes stay per-offset records.
        std::vector<uint32_t> flat, gflat;
        struct Group {
            uint32_t t;
            std::vector<uint32_t> used;  // union of the masks so far
            std::vector<std::pair<uint32_t, std::vector<uint32_t>>> items;
        };
        std::vector<Group> groups;
        uint32_t nrec = 0;
        for (auto &kv : qd) {
            uint32_t pm = 0;
            for (uint32_t t = 0; t < K; ++t)
                for (uint32_t w = 0; w < WS; ++w)
                    if (kv.second[(size_t)t * WS + w]) pm |= 1u << t;
            if (__builtin_popcount(pm) == 1) {
                const uint32_t t = __builtin_ctz(pm);
                std::vector<uint32_t> mk(kv.second.begin() + (size_t)t * WS, kv.second.begin() + (size_t)(t + 1) * WS);
                Group *dst = nullptr;
                for (auto &g : groups) {
                    if (g.t != t) continue;
                    bool disjoint = true;
                    for (uint32_t w = 0; w < WS && disjoint; ++w) disjoint = !(g.used[w] & mk[w]);
                    if (disjoint) {
                        dst = &g;
                        break;
                    }
                }
                if (!dst) {
                    groups.push_back(Group{t, std::vector<uint32_t>(WS, 0u), {}});
                    dst = &groups.back();
                }
                for (uint32_t w = 0; w < WS; ++w) dst->used[w] |= mk[w];
                dst->items.push_back({kv.first, mk});
                continue;
            }
            flat.push_back(kv.first);
            flat.push_back(pm);
            flat.insert(flat.end(), kv.second.begin(), kv.second.end());
            ++nrec;
        }
        for (auto &g : groups) {
            gflat.push_back(g.t);
            gflat.push_back((uint32_t)g.items.size());
            for (auto &it : g.items) {
                gflat.push_back(it.first);
                gflat.insert(gflat.end(), it.second.begin(), it.second.end());
            }
        }
        blob[H_NQD] = nrec;
        blob[H_OFF_QD] = append(flat);
        blob[H_NQG] = (uint32_t)groups.size();
        blob[H_OFF_QG] = append(gflat);
    }
    blob[H_OFF_COLIDX] = append(colidx);
    blob[H_OFF_COLENT] = append(colent);
    blob[H_OFF_THRINFO] = append(thrinfo);
    blob[H_OFF_THRTAB] = append(thrtab);
    {
        // real-energy records: ln |U| of every gate whose magnitude is not
        // constant, in gate order (the log-weight of a path is their sum)
        std::vector<uint32_t> re;
        uint32_t nre = 0;
        for (const GateC &g : gates) {
            if (g.const_mag) continue;
            std::vector<uint32_t> rec(RE_STRIDE, 0u);
            rec[0] = g.a;
            for (uint32_t j = 0; j < g.a; ++j) {
                rec[1 + j] = g.in_bits[j];
                rec[3 + j] = g.out_bits[j];
            }
            const uint32_t dim = 1u << g.a;
            for (uint32_t t = 0; t < dim * dim; ++t) {
                const double lm = g.mag[t] > 0.0 ? std::log(g.mag[t]) : 0.0;
                std::memcpy(&rec[8 + 2 * t], &lm, sizeof(double));
            }
            re.insert(re.end(), rec.begin(), rec.end());
            ++nre;
        }
        blob[H_NRE] = nre;
        blob[H_OFF_RE] = append(re);
    }
    {
        // toggle tables: row f of block j = XOR of the cones of the bits
        // 4j + t with bit t of f set, so one gather applies a block's flips
        const uint32_t nblk = (h + 3) / 4;
        const uint32_t TW = (WS + 3) & ~3u;
        std::vector<uint32_t> tog((size_t)nblk * 16 * TW, 0u);
        for (uint32_t j = 0; j < nblk; ++j)
            for (uint32_t f = 0; f < 16; ++f)
                for (uint32_t t = 0; t < 4; ++t)
                    if (((f >> t) & 1u) && 4 * j + t < h)
                        for (uint32_t w = 0; w < W; ++w) tog[((size_t)j * 16 + f) * TW + w] ^= cone[4 * j + t][w];
        blob[H_NBLK] = nblk;
        blob[H_TOGW] = TW;
        blob[H_OFF_TOG] = append(tog);
    }
    {
        // derived AND variables in layer order: the two lattice bits, then
        // the cone (WS words)
        std::vector<uint32_t> yr;
        for (uint32_t j = 0; j < ny; ++j) {
            yr.push_back(yvar[j][0]);
            yr.push_back(yvar[j][1]);
            std::vector<uint32_t> c = ycone[j];
            c.resize(WS, 0u);
            yr.insert(yr.end(), c.begin(), c.end());
        }
        blob[H_NY] = ny;
        blob[H_OFF_Y] = append(yr);
    }
    {
        // soft zeros: the four lattice bits of the gate (a one-qubit gate
        // repeats its bits: index bits 1 and 3 then copy bits 0 and 2, and
        // the mask is spread to the 4-bit index)
        std::vector<uint32_t> sr;
        uint32_t nsoft = 0;
        for (const GateC &g : gates) {
            bool any = false;
            for (bool v : g.soft) any = any || v;
            if (!any) continue;
            const uint32_t i1 = g.a == 2 ? g.in_bits[1] : g.in_bits[0];
            const uint32_t o1 = g.a == 2 ? g.out_bits[1] : g.out_bits[0];
            uint32_t mask = 0;
            for (uint32_t idx = 0; idx < 16; ++idx) {
                const uint32_t i = idx & 3u, o = idx >> 2;
                if (g.a == 1 && (((i ^ (i >> 1)) & 1u) || ((o ^ (o >> 1)) & 1u))) continue;
                const uint32_t t = g.a == 2 ? (o * 4 + i) : ((o & 1u) * 2 + (i & 1u));
                if (g.soft[t]) mask |= 1u << idx;
            }
            sr.insert(sr.end(), {g.in_bits[0], i1, g.out_bits[0], o1, mask});
            ++nsoft;
        }
        blob[H_NSOFT] = nsoft;
        blob[H_OFF_SOFT] = append(sr);
    }
    blob[H_THR_TOTAL] = (uint32_t)thrtab.size();
    blob[H_HBITS] = n + K;
    // pad so that kernels may read a few words past any array
    for (int i = 0; i < 64; ++i) blob.push_back(0);
    blob[H_TOTAL] = (uint32_t)blob.size();

    out.blob = std::move(blob);
    out.n = n;
    out.d = d;
    out.K = K;
    out.W = W;
    out.WS = WS;
    out.L = L;
    out.h = h;
    out.ny = ny;
    out.ncol = ncol;
    out.uniform = uniform;
    out.n_gates = G;
    out.nqd = (uint32_t)qd.size();
    out.circuit_id = D.circuit_id;
    out.has_z = true;
    out.Z = 1.0;
    for (const GateC &g : gates) {
        if (!g.has_col_sum) {
            out.has_z = false;
            break;
        }
        out.Z *= g.col_sum;
    }
    if (!out.has_z) out.Z = 0.0;
    return PBIT_OK;
}

}  // namespace pbit
