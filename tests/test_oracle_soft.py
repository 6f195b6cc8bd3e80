"""Pins of soft zeros (Appendix: e^(-J) in place of zero entries) in the
oracle: the controlled Hadamard written out, the compiled paths that avoid
every soft zero reproduce the statevector, the chain's binned law is the
exact path law (conditioning), and its binned fraction is the probability
of the valid paths under the e^(-J) sampling law."""
import math

import numpy as np
import pytest

from oracle import chain as och
from oracle import circuit as oc
from oracle import compile as ocomp
from oracle import estimator as oest
from oracle import exact
from workloads import circuits as wc


def test_controlled_hadamard_written_out():
    """CH with qubit 1 as control and qubit 0 as target: |c=1, t=0> goes to
    (|c=1, t=0> + |c=1, t=1>) / sqrt 2; |c=0, t=1> is unchanged."""
    r = 1 / math.sqrt(2)
    c = oc.from_dict(wc.circuit("ch", 2, 1, 1, [wc.ch(1, 1, 0)], 0b10))
    assert np.allclose(exact.statevector(c), [0, 0, r, r], atol=1e-15)
    c = oc.from_dict(wc.circuit("ch", 2, 1, 1, [wc.ch(1, 1, 0)], 0b01))
    assert np.allclose(exact.statevector(c), [0, 1, 0, 0], atol=1e-15)
    with pytest.raises(ocomp.CompileError):
        ocomp.compile_circuit(c)  # no soft_J: partial zeros are refused


@pytest.mark.parametrize("seed", range(6))
def test_valid_compiled_paths_reproduce_statevector(seed):
    circ = oc.from_dict(wc.random_clifford_t_ch(4, 6, 60 + seed, K=3))
    comp = ocomp.compile_circuit(circ, soft_J=3.0)
    amp = np.zeros(2 ** comp.n, dtype=complex)
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        assert (m > 0) == (not ocomp.violates(comp, x))
        if m > 0:
            amp[a] += m * np.exp(2j * math.pi * k / 2 ** comp.K)
    assert np.allclose(amp, exact.statevector(circ), atol=1e-12)


@pytest.mark.parametrize("J", [1.0, 3.0])
def test_binned_law_is_exact_and_fraction_is_valid_mass(J):
    circ = oc.from_dict(wc.random_clifford_t_ch(4, 6, 3, K=3))
    comp = ocomp.compile_circuit(circ, soft_J=J)
    chains, sweeps = 512, 200
    _, h = och.gibbs(comp, chains, 20, sweeps, seed=5, threads=8)
    T = int(h.sum())
    pm, _ = exact.magnitude_marginal(circ)
    assert oest.tv_path(h, pm) < 3 * oest.expected_iid_tv(pm, T)
    # the sampling law gives every free-bit assignment its e^(-J)-weight;
    # the binned fraction is the mass of the valid paths
    tot = valid = 0.0
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        w = ocomp.sampling_weight(comp, x)
        tot += w
        if m > 0:
            valid += w
    frac = valid / tot
    assert frac < 1.0
    assert T / (chains * sweeps) == pytest.approx(frac, abs=0.02)


def test_binning_violations_is_caught():
    """Planted mistake: binning the paths that meet a soft zero (their
    phase read as 0) leaves the binned law far from the exact one."""
    circ = oc.from_dict(wc.random_clifford_t_ch(4, 6, 3, K=3))
    comp = ocomp.compile_circuit(circ, soft_J=1.0)
    for g in comp.gates:
        g.soft = np.zeros_like(g.soft)
    _, h = och.gibbs(comp, 512, 20, 200, seed=5, threads=8)
    pm, _ = exact.magnitude_marginal(circ)
    assert oest.tv_path(h, pm) > 10 * oest.expected_iid_tv(pm, int(h.sum()))
