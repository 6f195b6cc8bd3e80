"""Monte Carlo estimator of the amplitudes (test infrastructure only).

Eq. (U343)/(U344): U_{alpha,beta} = sum_C p_C W_C with W_C = psi_C / p_C.
With p_C = |psi_C| / Z (Eq. (weightedS)) every sample carries
W_C = Z exp(2 pi i k / 2^K), so Eq. (U23) becomes
    A_alpha = Z / T * sum_k c_{alpha,k} omega^k,   omega = exp(2 pi i / 2^K),
where c_{alpha,k} counts the samples binned at output alpha, phase k.
Eq. (U26)/(U30): the standard deviation of the estimate is
std({W_C}) / sqrt(T); it is evaluated here per real and imaginary part from
the counts (or from exact bin probabilities).
Fig. 2 step 4: the L2 mode divides every bin by the root of the sum of the
squared bin moduli instead of using Z.
"""
from __future__ import annotations

import math

import numpy as np


def _omega(K):
    k = np.arange(2 ** K)
    ang = 2.0 * math.pi * k / (2 ** K)
    cs, sn = np.cos(ang), np.sin(ang)
    # quarter turns are exact zeros of cos / sin
    cs[np.abs(cs) < 1e-15] = 0.0
    sn[np.abs(sn) < 1e-15] = 0.0
    return cs, sn


def amplitudes(counts, Z, T=None):
    """counts[alpha, k] (integers) -> (amp complex[2^n], sig_re, sig_im)."""
    counts = np.asarray(counts, dtype=np.float64)
    K = int(round(math.log2(counts.shape[1])))
    T = float(counts.sum()) if T is None else float(T)
    cs, sn = _omega(K)
    f = counts / T                         # empirical bin frequencies
    mre = f @ cs
    mim = f @ sn
    amp = Z * (mre + 1j * mim)
    var_re = Z * Z * (f @ (cs * cs) - mre * mre) / T
    var_im = Z * Z * (f @ (sn * sn) - mim * mim) / T
    return amp, np.sqrt(np.maximum(var_re, 0.0)), np.sqrt(np.maximum(var_im, 0.0))


def amplitudes_l2(counts):
    """Fig. 2 step 4: bin sums divided by their L2 norm."""
    counts = np.asarray(counts, dtype=np.float64)
    K = int(round(math.log2(counts.shape[1])))
    cs, sn = _omega(K)
    A = counts @ cs + 1j * (counts @ sn)
    nrm = math.sqrt(float(np.sum(np.abs(A) ** 2)))
    return A / nrm if nrm > 0 else A


def exact_sigma(prob, Z, T):
    """Per-component sigma from exact bin probabilities prob[alpha, k]."""
    prob = np.asarray(prob, dtype=np.float64)
    K = int(round(math.log2(prob.shape[1])))
    cs, sn = _omega(K)
    mre, mim = prob @ cs, prob @ sn
    vre = Z * Z * (prob @ (cs * cs) - mre * mre) / T
    vim = Z * Z * (prob @ (sn * sn) - mim * mim) / T
    return np.sqrt(np.maximum(vre, 0)), np.sqrt(np.maximum(vim, 0))


def tv_path(counts, p_mag):
    """Total variation between the sampled output marginal and the exact
    magnitude marginal of Eq. (weightedS)."""
    counts = np.asarray(counts, dtype=np.float64)
    emp = counts.sum(axis=1) / counts.sum()
    return 0.5 * float(np.abs(emp - np.asarray(p_mag)).sum())


def tv_born(amp, psi):
    p = np.abs(amp) ** 2
    p = p / p.sum() if p.sum() > 0 else p
    q = np.abs(psi) ** 2
    return 0.5 * float(np.abs(p - q).sum())


def expected_iid_tv(p_mag, T):
    """E TV of an iid empirical marginal of size T (normal approximation)."""
    p = np.asarray(p_mag, dtype=np.float64)
    return 0.5 * float(np.sum(np.sqrt(2.0 * p * (1.0 - p) / (math.pi * T))))


def z_gate(amp, sig_re, sig_im, psi, zmax_count_p=6.3e-5):
    """The 4-sigma acceptance rule across many amplitude components:
    (i) the number of |z| > 4 stays below the 99.9% binomial quantile,
    (ii) max |z| stays below the Bonferroni bound at 0.5% family-wise,
    (iii) sum z^2 stays within 4 sqrt(2 m) of its mean m.
    Components with zero sigma must match exactly (to 1e-9 relative).
    Returns (ok, info)."""
    from scipy import stats
    zs = []
    exact_bad = 0
    for est, sg, ex in ((amp.real, sig_re, psi.real), (amp.imag, sig_im, psi.imag)):
        for e, s, x in zip(est, sg, ex):
            if s == 0.0:
                if abs(e - x) > 1e-9 * max(1.0, abs(x)):
                    exact_bad += 1
                continue
            zs.append((e - x) / s)
    zs = np.array(zs)
    m = len(zs)
    if m == 0:
        return exact_bad == 0, dict(m=0, exact_bad=exact_bad)
    n_over = int(np.sum(np.abs(zs) > 4.0))
    lim_over = int(stats.binom.ppf(0.999, m, zmax_count_p))
    zmax = float(np.max(np.abs(zs)))
    lim_max = float(stats.norm.isf(0.005 / (2.0 * m)))
    chi2 = float(np.sum(zs * zs))
    ok = (n_over <= lim_over and zmax <= max(lim_max, 4.0) and abs(chi2 - m) <= 4.0 * math.sqrt(2.0 * m)
          and exact_bad == 0)
    return ok, dict(m=m, n_over=n_over, lim_over=lim_over, zmax=zmax, lim_max=lim_max,
                    chi2=chi2, exact_bad=exact_bad)
