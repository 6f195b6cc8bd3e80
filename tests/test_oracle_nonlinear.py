"""Pins of the oracle's three-qubit permutation gates (Appendix, CCNOT):
the Toffoli's truth table written out, compiled paths of circuits with
Toffoli and Peres gates against the statevector, the gate-by-gate lattice
against the cone lattice on affine circuits, and the chain's support."""
import math

import numpy as np
import pytest

from oracle import chain as och
from oracle import circuit as oc
from oracle import compile as ocomp
from oracle import estimator as oest
from oracle import exact
from workloads import circuits as wc


def test_toffoli_truth_table():
    """s_t' = s_t XOR (s_c1 AND s_c2), controls unchanged, for all eight
    basis inputs (the Appendix's CCNOT), through the statevector."""
    for t in (0, 1):
        for a in (0, 1):
            for b in (0, 1):
                inp = t | (a << 1) | (b << 2)
                c = oc.from_dict(wc.circuit("tof", 3, 1, 1, [wc.toffoli(1, 0, 1, 2)], inp))
                psi = exact.statevector(c)
                want = (t ^ (a & b)) | (a << 1) | (b << 2)
                assert abs(psi[want] - 1.0) < 1e-15 and np.abs(psi).sum() == pytest.approx(1.0)


def _compiled_amplitudes(comp):
    amp = np.zeros(2 ** comp.n, dtype=complex)
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        amp[a] += m * np.exp(2j * math.pi * k / 2 ** comp.K)
    return amp


@pytest.mark.parametrize("seed", range(8))
def test_compiled_paths_with_toffoli_reproduce_statevector(seed):
    """Random Clifford+T circuits with Toffoli and Peres gates: summing
    |psi_C| e^{2 pi i k / 2^K} over the 2^h free-bit assignments, each
    lattice evaluated gate by gate, gives the statevector (and the
    brute-force path sum over all 2^(n d) configurations)."""
    c = oc.from_dict(wc.random_clifford_t_toffoli(4, 4, 300 + seed, K=3, p3=0.5))
    comp = ocomp.compile_circuit(c)
    assert comp.nonlinear == any(g.arity == 3 for g in c.gates)
    psi = exact.statevector(c)
    assert np.allclose(_compiled_amplitudes(comp), psi, atol=1e-12)
    assert np.allclose(exact.path_sum(c), psi, atol=1e-12)


@pytest.mark.parametrize("name", ["tiny", "rct12"])
def test_forward_lattice_equals_cone_lattice(name):
    """On affine circuits the gate-by-gate lattice equals the constant
    lattice with the cones of the set free bits flipped."""
    comp = ocomp.compile_circuit(oc.from_dict(wc.workload_circuit(name)))
    rng = np.random.default_rng(1)
    for _ in range(20):
        f = rng.integers(0, 2, comp.h).tolist()
        assert (ocomp.forward_lattice(comp, f) == ocomp.lattice_from_free(comp, f)).all()


def test_nonlinear_chain_support_and_law():
    """A Toffoli circuit's chains visit only valid paths and their output
    law matches the exact magnitude marginal (TV at the i.i.d. level)."""
    c = wc.random_clifford_t_toffoli(4, 4, 7, K=3, p3=0.9)
    circ = oc.from_dict(c)
    comp = ocomp.compile_circuit(circ)
    assert comp.nonlinear
    st, h = och.gibbs(comp, 32, 2, 100, seed=3)
    pm, Z = exact.magnitude_marginal(circ)
    assert oest.tv_path(h, pm) < 3 * oest.expected_iid_tv(pm, 3200)
    valid = {tuple(ocomp.pack_words(x, comp.W)) for f, x, m, k, a in ocomp.enumerate_free(comp)}
    assert all(tuple(w) in valid for w in st)


def test_nonuniform_nonlinear_is_rejected():
    """Non-affine gates with a gate of non-constant magnitude: the compile
    refuses (the conditionals would need the lattice re-evaluated)."""
    g = [wc.gate1(1, 0, "RH", wc.mat_rh(math.pi / 8)), wc.toffoli(2, 0, 1, 2)]
    with pytest.raises(ocomp.CompileError):
        ocomp.compile_circuit(oc.from_dict(wc.circuit("nu", 3, 2, 1, g, 0)))
