"""Pins of the oracle's estimator (Eqs. (U343), (U23), (U26), (U30) and the
L2 mode of Fig. 2 step 4) to values fixed by the paper and by hand.

Each test feeds the estimator the counts a run would produce at exact
expectation, c_{alpha,k} = T * P(alpha, k), with P written out by hand (the
tiny circuit's four equally likely paths, the even-d Hadamard chain's
uniform paths with the peak height of Sec. 4) or enumerated over the
compiled lattice of small random circuits.  At expectation the exact-Z
estimate is psi itself, the L2-normalised bin sums are psi / |psi| = psi,
and the per-component sigma takes the closed forms of Eq. (stdT) and of
the tiny circuit.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import circuit as oc
from oracle import compile as ocomp
from oracle import estimator as oest
from oracle import exact
from workloads import circuits as wc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def tiny_expected_counts(T):
    """The n=3 circuit's four paths (one per output 0, 2, 5, 7, magnitude
    1/2 each) carry the phase bins of the golden file: each gets T/4."""
    g = json.load(open(os.path.join(GOLD, "tiny_n3_d5.json")))
    counts = np.zeros((8, 2 ** g["K"]))
    for a, k in g["phase_bins"].items():
        counts[int(a), k] = T / 4.0
    want = np.zeros(8, dtype=complex)
    for a, (re, im) in g["amplitudes"].items():
        want[int(a)] = complex(re, im)
    return counts, want, g["Z"]


def hadamard_expected_counts(d, T):
    """Even-d Hadamard chain (Sec. 4, 'Sign problem'), K = 1: every path has
    magnitude 2^(-d/2) and sign +-1, half of them end in each output.  At the
    correct output 0 the signed fraction is the peak height 2^(-d/2), so
    P(0, +) = (1/2 + 2^(-d/2)) / 2 and P(0, -) = (1/2 - 2^(-d/2)) / 2; at the
    wrong output 1 both signs have probability 1/4.  Z = 2^(d/2)."""
    p = 2.0 ** (-d / 2)
    counts = T * np.array([[(0.5 + p) / 2, (0.5 - p) / 2], [0.25, 0.25]])
    return counts, np.array([1.0, 0.0], dtype=complex), 2.0 ** (d / 2)


def test_tiny_at_expectation_exact_z_and_l2_give_psi():
    T = 2048000
    counts, want, Z = tiny_expected_counts(T)
    amp, sre, sim = oest.amplitudes(counts, Z)
    assert np.allclose(amp, want, atol=1e-14)
    assert np.allclose(oest.amplitudes_l2(counts), want, atol=1e-14)
    # sigma from the counts: outputs 0 and 2 carry W = Z with probability
    # 1/4, so Var Re = (Z^2/4 - 1/4) / T = 3 / (4T); outputs 5 and 7 carry
    # W = Z e^{+-i pi/4}: Var Re = Var Im = (Z^2/8 - 1/8) / T = 0.375 / T
    for a in (0, 2):
        assert sre[a] == pytest.approx(math.sqrt(3.0 / (4 * T)), rel=1e-12)
        assert sim[a] == 0.0
    for a in (5, 7):
        assert sre[a] == pytest.approx(math.sqrt(0.375 / T), rel=1e-12)
        assert sim[a] == pytest.approx(math.sqrt(0.375 / T), rel=1e-12)
    for a in (1, 3, 4, 6):
        assert sre[a] == 0.0 and sim[a] == 0.0


@pytest.mark.parametrize("d", [2, 4, 6, 8, 10])
def test_hadamard_chain_at_expectation(d):
    """The exact-Z estimate at expectation is |0>; its sigma on the wrong
    output is Eq. (stdT), 2^(d/2) / sqrt(2T); the L2 mode gives |0>."""
    T = 10 ** 7
    counts, want, Z = hadamard_expected_counts(d, T)
    amp, sre, sim = oest.amplitudes(counts, Z)
    assert np.allclose(amp, want, atol=1e-12)
    assert sre[1] == pytest.approx(2.0 ** (d / 2) / math.sqrt(2 * T), rel=1e-12)
    # on the correct output: W = +-Z, E W = 1, E W^2 = Z^2 / 2
    assert sre[0] == pytest.approx(math.sqrt((Z * Z / 2 - 1.0) / T), rel=1e-12)
    assert np.all(sim == 0.0)
    l2 = oest.amplitudes_l2(counts)
    assert np.allclose(l2, want, atol=1e-12)


@pytest.mark.parametrize("d", [4, 8])
def test_hadamard_chain_counts_recover_stdT_when_T_is_implicit(d):
    """amplitudes() takes T from the counts when T is not given."""
    counts, _, Z = hadamard_expected_counts(d, 10 ** 6)
    _, sre, _ = oest.amplitudes(counts, Z)
    assert sre[1] == pytest.approx(2.0 ** (d / 2) / math.sqrt(2e6), rel=1e-12)


def _enumerated_counts(circ, T):
    comp = ocomp.compile_circuit(circ)
    K = circ.K
    counts = np.zeros((2 ** circ.n, 2 ** K))
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        counts[a, k] += T * m / comp.Z
    return counts, comp.Z


@pytest.mark.parametrize("seed", range(8))
def test_random_circuits_at_expectation_match_statevector(seed):
    """Eq. (U343): the estimator is unbiased, so exact-expectation counts
    (each path's bin gets T |psi_C| / Z) reproduce the statevector in exact-Z
    mode and psi / |psi| = psi in the L2 mode, for inputs beta != 0 too."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 4))
    d = int(rng.integers(2, 5))
    c = wc.random_asymmetric(n, d, seed, K=3) if seed % 2 else wc.random_clifford_t(n, d, seed, K=3)
    c = dict(c, input=int(rng.integers(0, 2 ** n)))
    circ = oc.from_dict(c)
    counts, Z = _enumerated_counts(circ, 1e9)
    psi = exact.statevector(circ)
    amp, _, _ = oest.amplitudes(counts, Z)
    assert np.allclose(amp, psi, atol=1e-12)
    assert np.allclose(oest.amplitudes_l2(counts), psi, atol=1e-12)


def test_l2_mode_is_scale_free_and_unit_norm():
    """Fig. 2 step 4 divides by the L2 norm of the bin sums: the result has
    norm 1 and does not depend on the number of samples."""
    counts, _, _ = tiny_expected_counts(4000)
    a = oest.amplitudes_l2(counts)
    b = oest.amplitudes_l2(counts * 37)
    assert np.linalg.norm(a) == pytest.approx(1.0, abs=1e-14)
    assert np.allclose(a, b, atol=1e-15)
