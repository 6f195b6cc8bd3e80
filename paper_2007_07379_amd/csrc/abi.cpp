// C ABI of the library: handle lifecycle, argument checking, run planning
// (sweep groups, histogram privatisation, graph replay) and FP64 amplitude
// recovery.  Every public function returns a status; no exception crosses
// the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pbit.h"
#include "blob.h"
#include "compile.h"
#include "gibbs.h"
#include "runtime.h"
#include "shor.h"

namespace pbit {

thread_local std::string g_last_error;

pbit_status set_error(pbit_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

pbit_status hip_error(hipError_t e, const char *what) {
    return set_error(PBIT_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace pbit

using namespace pbit;

extern "C" {

const char *pbit_last_error(void) { return g_last_error.c_str(); }

static pbit_status shor_check(const pbit_shor_cfg *cfg) {
    if (!cfg) return set_error(PBIT_E_INVALID_ARG, "NULL cfg");
    if (cfg->N < 3 || cfg->N >= (1ull << 31)) return set_error(PBIT_E_INVALID_ARG, "N must be in [3, 2^31)");
    if (cfg->a < 2 || cfg->a >= cfg->N) return set_error(PBIT_E_INVALID_ARG, "a must be in (1, N)");
    if (cfg->n < 1 || cfg->n > 30) return set_error(PBIT_E_INVALID_ARG, "n must be in [1, 30]");
    if (cfg->T < 1 || cfg->T > (1u << 22)) return set_error(PBIT_E_INVALID_ARG, "T must be in [1, 2^22]");
    return PBIT_OK;
}

pbit_status pbit_shor_work_bytes(const pbit_shor_cfg *cfg, size_t *bytes) {
    const pbit_status st = shor_check(cfg);
    if (st != PBIT_OK) return st;
    if (!bytes) return set_error(PBIT_E_INVALID_ARG, "NULL bytes");
    *bytes = (size_t)shor_pad(cfg->T) * sizeof(uint64_t);
    return PBIT_OK;
}

pbit_status pbit_shor_run(const pbit_shor_cfg *cfg, float *d_P, void *d_work, void *hip_stream) {
    const pbit_status st = shor_check(cfg);
    if (st != PBIT_OK) return st;
    if (!d_P || !d_work) return set_error(PBIT_E_INVALID_ARG, "NULL d_P or d_work");
    if ((uintptr_t)d_work % 8) return set_error(PBIT_E_INVALID_ARG, "d_work must be 8-byte aligned");
    const hipError_t e = launch_shor(cfg->N, cfg->a, cfg->n, cfg->T, cfg->seed, d_P, (uint64_t *)d_work,
                                     (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_error(e, "column sampling launch");
    return PBIT_OK;
}

pbit_status pbit_compile_circuit(const pbit_circuit_desc *descs, uint32_t n_circuits, pbit_circuit *out) {
    if (!out) return set_error(PBIT_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!descs || n_circuits == 0) return set_error(PBIT_E_INVALID_ARG, "no circuits");
    try {
        auto *h = new pbit_circuit_s();
        h->circuits.resize(n_circuits);
        uint64_t hoff = 0;
        for (uint32_t i = 0; i < n_circuits; ++i) {
            std::string err;
            pbit_status st = compile_one(descs[i], h->circuits[i], err);
            if (st != PBIT_OK) {
                delete h;
                return set_error(st, "circuit " + std::to_string(i) + ": " + err);
            }
            h->hist_off.push_back(hoff);
            hoff += 1ull << (h->circuits[i].n + h->circuits[i].K);
        }
        h->hist_total = hoff;
        *out = h;
        return PBIT_OK;
    } catch (const std::bad_alloc &) {
        return set_error(PBIT_E_OOM, "host allocation failed");
    }
}

void pbit_circuit_free(pbit_circuit c) { delete c; }

uint32_t pbit_circuit_count(pbit_circuit c) { return c ? (uint32_t)c->circuits.size() : 0u; }

pbit_status pbit_circuit_info_get(pbit_circuit c, uint32_t idx, pbit_circuit_info *out) {
    if (!c || !out || idx >= c->circuits.size()) return set_error(PBIT_E_INVALID_ARG, "bad handle or index");
    const CompiledCircuit &k = c->circuits[idx];
    std::memset(out, 0, sizeof(*out));
    out->n = k.n;
    out->d = k.d;
    out->K = k.K;
    out->W = k.W;
    out->L = k.L;
    out->h = k.h;
    out->n_colours = k.ncol;
    out->uniform = k.uniform ? 1u : 0u;
    out->n_gates = k.n_gates;
    out->n_quad_offsets = k.nqd;
    out->hist_bins = 1u << (k.n + k.K);
    out->circuit_id = k.circuit_id;
    out->has_exact_z = k.has_z ? 1 : 0;
    out->Z = k.Z;
    out->hist_offset = c->hist_off[idx];
    return PBIT_OK;
}

pbit_status pbit_circuit_export(pbit_circuit c, uint32_t idx, uint32_t *buf, size_t *len) {
    if (!c || !len || idx >= c->circuits.size()) return set_error(PBIT_E_INVALID_ARG, "bad handle or index");
    const auto &b = c->circuits[idx].blob;
    if (buf) {
        if (*len < b.size()) return set_error(PBIT_E_INVALID_ARG, "buffer too small");
        std::memcpy(buf, b.data(), b.size() * sizeof(uint32_t));
    }
    *len = b.size();
    return PBIT_OK;
}

pbit_status pbit_gibbs_run(pbit_circuit c, const pbit_gibbs_cfg *cfg, uint32_t *d_state, uint32_t *d_hist,
                           void *hip_stream) {
    return run_gibbs(c, cfg, d_state, d_hist, (hipStream_t)hip_stream);
}

pbit_status pbit_sync(void *hip_stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
    return PBIT_OK;
}

pbit_status pbit_amplitudes(pbit_circuit c, uint32_t idx, const uint64_t *counts, uint64_t T, int mode,
                            double *amp_re, double *amp_im, double *sig_re, double *sig_im) {
    if (!c || idx >= c->circuits.size() || !counts || !amp_re || !amp_im)
        return set_error(PBIT_E_INVALID_ARG, "bad handle, index or NULL buffer");
    if (mode != PBIT_NORM_EXACT_Z && mode != PBIT_NORM_L2) return set_error(PBIT_E_INVALID_ARG, "bad mode");
    const CompiledCircuit &k = c->circuits[idx];
    if (mode == PBIT_NORM_EXACT_Z && !k.has_z)
        return set_error(PBIT_E_MODE_UNAVAILABLE, "exact Z needs constant gate column sums");
    const uint32_t nk = 1u << k.K;
    const uint64_t na = 1ull << k.n;
    if (mode == PBIT_NORM_EXACT_Z && T == 0) return set_error(PBIT_E_INVALID_ARG, "T == 0");
    // omega^k with exact zeros at quarter turns
    std::vector<double> cs(nk), sn(nk);
    for (uint32_t j = 0; j < nk; ++j) {
        const double ang = 2.0 * M_PI * (double)j / (double)nk;
        cs[j] = std::cos(ang);
        sn[j] = std::sin(ang);
        if (std::fabs(cs[j]) < 1e-15) cs[j] = 0.0;
        if (std::fabs(sn[j]) < 1e-15) sn[j] = 0.0;
    }
    if (mode == PBIT_NORM_EXACT_Z) {
        // Eq. (U23) with W_C = Z omega^k; Eq. (U26) per component
        const double Z = k.Z, Tf = (double)T;
        for (uint64_t a = 0; a < na; ++a) {
            const uint64_t *row = counts + a * nk;
            double mr = 0, mi = 0, m2r = 0, m2i = 0;
            for (uint32_t j = 0; j < nk; ++j) {
                const double f = (double)row[j] / Tf;
                mr += f * cs[j];
                mi += f * sn[j];
                m2r += f * cs[j] * cs[j];
                m2i += f * sn[j] * sn[j];
            }
            amp_re[a] = Z * mr;
            amp_im[a] = Z * mi;
            if (sig_re) sig_re[a] = std::sqrt(std::max(0.0, Z * Z * (m2r - mr * mr) / Tf));
            if (sig_im) sig_im[a] = std::sqrt(std::max(0.0, Z * Z * (m2i - mi * mi) / Tf));
        }
    } else {
        // Fig. 2 step 4: divide every bin by the L2 norm of all bins
        double nrm2 = 0;
        for (uint64_t a = 0; a < na; ++a) {
            const uint64_t *row = counts + a * nk;
            double br = 0, bi = 0;
            for (uint32_t j = 0; j < nk; ++j) {
                br += (double)row[j] * cs[j];
                bi += (double)row[j] * sn[j];
            }
            amp_re[a] = br;
            amp_im[a] = bi;
            nrm2 += br * br + bi * bi;
        }
        const double inv = nrm2 > 0 ? 1.0 / std::sqrt(nrm2) : 0.0;
        for (uint64_t a = 0; a < na; ++a) {
            amp_re[a] *= inv;
            amp_im[a] *= inv;
            if (sig_re) sig_re[a] = 0.0;
            if (sig_im) sig_im[a] = 0.0;
        }
    }
    return PBIT_OK;
}

}  // extern "C"
