"""Pins of the oracle's exact layer (statevector, path sum, compile) to the
paper and to mathematics other than the oracle itself."""
import cmath
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


def _circ(c):
    return oc.from_dict(c)


def small_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 4))
    d = int(rng.integers(1, 5 if n < 3 else 4))
    return _circ(wc.random_clifford_t(n, d, seed, K=3))


def small_asym(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 4))
    d = int(rng.integers(1, 5 if n < 3 else 4))
    return _circ(wc.random_asymmetric(n, d, seed, K=3))


@pytest.mark.parametrize("seed", range(18))
def test_statevector_equals_path_sum_and_dense(seed):
    """Eq. (U) as a matrix product and Eq. (path) as an explicit sum over
    every Feynman path are the same number (exact identity); seeds >= 12 use
    circuits with non-symmetric gates."""
    c = small_random(seed) if seed < 12 else small_asym(seed)
    sv = exact.statevector(c)
    ps = exact.path_sum(c)
    dense = exact.dense_unitary(c)[:, c.input]
    assert np.allclose(sv, ps, atol=1e-12)
    assert np.allclose(sv, dense, atol=1e-12)
    assert abs(np.linalg.norm(sv) - 1.0) < 1e-12


def test_tiny_amplitudes_and_phase_bins():
    g = json.load(open(os.path.join(GOLD, "tiny_n3_d5.json")))
    c = _circ(wc.tiny_ghz_t())
    sv = exact.statevector(c)
    want = np.zeros(8, dtype=complex)
    for k, (re, im) in g["amplitudes"].items():
        want[int(k)] = complex(re, im)
    assert np.allclose(sv, want, atol=1e-12)
    assert np.allclose(exact.path_sum(c), want, atol=1e-12)
    comp = ocomp.compile_circuit(c)
    assert comp.h == g["free_bits"]
    assert comp.Z == pytest.approx(g["Z"], rel=1e-12)
    # every path of the compiled lattice lands on one of the four outputs
    # with the phase bin of its amplitude
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        assert str(a) in g["phase_bins"]
        assert k == g["phase_bins"][str(a)]
        assert m == pytest.approx(0.5)


@pytest.mark.parametrize("inp", ["1", "5"])
def test_tiny_nonzero_inputs(inp):
    """The tiny circuit on inputs beta = 1 and 5, worked by hand (golden
    file): the statevector, the path sum, the dense column beta and every
    path of the compiled lattice (clamped to beta on layer 0) agree with it."""
    g = json.load(open(os.path.join(GOLD, "tiny_n3_d5_inputs.json")))
    case = g["inputs"][inp]
    c = _circ(dict(wc.tiny_ghz_t(), input=int(inp)))
    want = np.zeros(8, dtype=complex)
    for k, (re, im) in case["amplitudes"].items():
        want[int(k)] = complex(re, im)
    assert np.allclose(exact.statevector(c), want, atol=1e-12)
    assert np.allclose(exact.path_sum(c), want, atol=1e-12)
    assert np.allclose(exact.dense_unitary(c)[:, int(inp)], want, atol=1e-12)
    comp = ocomp.compile_circuit(c)
    assert comp.h == g["free_bits"] and comp.Z == pytest.approx(g["Z"], rel=1e-12)
    seen = set()
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        assert [x[q] for q in range(3)] == [(int(inp) >> q) & 1 for q in range(3)]
        assert k == case["phase_bins"][str(a)]
        assert m == pytest.approx(0.5)
        seen.add(a)
    assert seen == {int(a) for a in case["phase_bins"]}


@pytest.mark.parametrize("seed", range(12))
def test_nonzero_inputs_statevector_path_sum_dense_and_compile(seed):
    """Inputs beta != 0 (1, 5 and all ones, reduced mod 2^n): Eq. (U) as a
    matrix product, Eq. (path) as an explicit sum, the dense unitary's
    column beta and the compiled lattice's path sum are the same vector."""
    c = small_random(seed) if seed % 2 else small_asym(seed)
    for beta in sorted({1 % 2 ** c.n, 5 % 2 ** c.n, 2 ** c.n - 1}):
        cb = oc.Circuit(c.n, c.d, c.K, beta, c.gates, c.name)
        sv = exact.statevector(cb)
        assert np.allclose(sv, exact.path_sum(cb), atol=1e-12), beta
        assert np.allclose(sv, exact.dense_unitary(cb)[:, beta], atol=1e-12), beta
        comp = ocomp.compile_circuit(cb)
        assert np.allclose(compiled_amplitudes(comp), sv, atol=1e-12), beta


def test_hadamard_d2_worked_example():
    """Sec. 4, Fig. 3: four equal-magnitude paths, 0->1->1 has the opposite
    phase; output 0 collects 2, output 1 collects 0."""
    g = json.load(open(os.path.join(GOLD, "hadamard_d2.json")))
    c = _circ(wc.hadamard_chain(2, K=1))
    _, paths = exact.path_sum(c, return_paths=True)
    got = {tuple(s): w for s, w in paths}
    assert len(got) == 4
    for p in g["paths"]:
        w = got[tuple(p["layers"])]
        assert abs(w) == pytest.approx(g["path_magnitude"])
        assert np.sign(w.real) == p["sign"]
    comp = ocomp.compile_circuit(c)
    sums = {0: 0, 1: 0}
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        sums[a] += 1 if k == 0 else -1
    assert sums == {int(k): v for k, v in g["phase_sum"].items()}


@pytest.mark.parametrize("d", [2, 4, 6, 8, 10])
def test_peak_height_even_hadamard_chain(d):
    """Sec. 4 'Sign problem': with uniform sampling the net signed count at
    the correct output, as a fraction of all samples, is 2^(-d/2)."""
    comp = ocomp.compile_circuit(_circ(wc.hadamard_chain(d, K=1)))
    assert comp.h == d
    net = 0
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        if a == 0:
            net += 1 if k == 0 else -1
    assert net / 2 ** comp.h == pytest.approx(2.0 ** (-d / 2))


@pytest.mark.parametrize("d", [2, 4, 6, 8])
def test_sigma_wrong_output_eq_stdT(d):
    """Eq. (stdT): on the wrong output of an even-d Hadamard chain the
    estimator's standard deviation is 2^(d/2) / sqrt(2T)."""
    comp = ocomp.compile_circuit(_circ(wc.hadamard_chain(d, K=1)))
    prob = np.zeros((2, 2))
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        prob[a, k] += 1.0 / 2 ** comp.h
    T = 10 ** 6
    sre, sim = oest.exact_sigma(prob, comp.Z, T)
    assert comp.Z == pytest.approx(2.0 ** (d / 2))
    assert sre[1] == pytest.approx(2.0 ** (d / 2) / math.sqrt(2 * T), rel=1e-12)
    assert sim[1] == 0.0


def test_tiny_sigma_closed_form():
    """Config n=3: outputs 0 and 2 have W_C = Z = 2 with probability 1/4
    each, so Var Re A = (4 - 1) / (4 T)."""
    comp = ocomp.compile_circuit(_circ(wc.tiny_ghz_t()))
    prob = np.zeros((8, 8))
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        prob[a, k] += 0.25
    T = 2048000
    sre, _ = oest.exact_sigma(prob, comp.Z, T)
    assert sre[0] == pytest.approx(math.sqrt(3.0 / (4 * T)), rel=1e-12)
    assert sre[5] == pytest.approx(math.sqrt(0.375 / T), rel=1e-12)


def _eb_energy(U, s_out, s_in):
    """Eq. (EB) with principal complex logs."""
    a1, b1, c1, A1 = U[0, 0], U[0, 1], U[1, 0], U[1, 1]
    L = cmath.log
    return (-L(a1) + s_out * L(a1 / c1) + s_in * L(a1 / b1)
            + s_in * s_out * L(b1 * c1 / (a1 * A1)))


@pytest.mark.parametrize("seed", range(6))
def test_table_orientation_matches_eq_EB(seed):
    """The oracle's magnitude/phase table entry at (out, in) reproduces
    exp(-E) of the Boolean form Eq. (EB) at (s^(d), s^(d-1)) = (out, in);
    a transposed table fails for non-symmetric U."""
    rng = np.random.default_rng(seed)
    K = 3
    mags = rng.uniform(0.2, 1.0, size=(2, 2))
    ks = rng.integers(0, 2 ** K, size=(2, 2))
    U = mags * np.exp(2j * np.pi * ks / 2 ** K)
    circ = oc.Circuit(1, 1, K, 0, [oc.Gate(1, [0], U)])
    g = ocomp.compile_circuit(circ).gates[0]
    for o in (0, 1):
        for i in (0, 1):
            val = cmath.exp(-_eb_energy(U, o, i))
            tab = g.mag[o * 2 + i] * cmath.exp(2j * math.pi * g.ph[o * 2 + i] / 2 ** K)
            assert abs(val - tab) < 1e-12
            assert abs(val - U[o, i]) < 1e-12


def test_eq2E_hadamard_energy():
    """Eq. (eq2E): for two Hadamards the imaginary energy is
    i pi (s1 s2 + s2 s3); the table phases sum to pi (s1 s2 + s2 s3)."""
    comp = ocomp.compile_circuit(_circ(wc.hadamard_chain(2, K=1)))
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        s1, s2, s3 = int(x[0]), int(x[1]), int(x[2])
        assert k == (s1 * s2 + s2 * s3) % 2
    # a1 = b1 = c1 = -A1 = 1 in Eq. (EB): E = i pi s s'
    U = np.array([[1, 1], [1, -1]], dtype=complex)
    for o in (0, 1):
        for i in (0, 1):
            e = _eb_energy(U, o, i)
            assert abs(cmath.exp(-e) - cmath.exp(-1j * math.pi * o * i)) < 1e-12


def _one_gate(U, arity, n=2, K=3, inp=0):
    qubits = [0] if arity == 1 else [0, 1]
    return ocomp.compile_circuit(oc.Circuit(n, 1, K, inp, [oc.Gate(1, qubits, U)]))


@pytest.mark.parametrize("inp", range(4))
def test_appendix_cnot_is_xor(inp):
    """Appendix, CNOT: with the paper's matrix (qubit 2 controls),
    s1' = s1 XOR s2, s2' = s2, E = 0; no free p-bit is created."""
    U = np.array(wc.mat_cnot_tc()[0], dtype=complex)
    comp = _one_gate(U, 2, inp=inp)
    assert comp.gates[0].kind == "derived" and comp.h == 0
    s1, s2 = inp & 1, (inp >> 1) & 1
    assert comp.const[2] == s1 ^ s2 and comp.const[3] == s2
    assert comp.gates[0].ph.max() == 0


@pytest.mark.parametrize("inp", [0, 1])
def test_appendix_not_and_rz(inp):
    """Appendix: Pauli-X sets s' = 1 - s with E = 0; Rz(gamma) keeps s' = s
    and carries U = exp(-i gamma (1 - 2 s) / 2) (from -ln U directly)."""
    comp = _one_gate(np.array(wc.mat_x()[0], dtype=complex), 1, n=1, inp=inp)
    assert comp.gates[0].kind == "derived" and comp.const[1] == 1 - inp
    gamma = math.pi / 2
    re, im = wc.mat_rz(gamma)
    U = np.array(re) + 1j * np.array(im)
    comp = _one_gate(U, 1, n=1, K=3, inp=inp)
    g = comp.gates[0]
    assert g.kind == "copy" and comp.const[1] == inp
    k = g.ph[inp * 2 + inp]
    val = cmath.exp(2j * math.pi * k / 8)
    assert abs(val - cmath.exp(-1j * gamma * (1 - 2 * inp) / 2)) < 1e-12


def test_appendix_exchange_j12_copies():
    gamma = math.pi / 2
    e = cmath.exp(1j * gamma / 2)
    U = np.diag([e, e.conjugate(), e.conjugate(), e])
    comp = _one_gate(U, 2, K=3, inp=3)
    assert comp.gates[0].kind == "copy" and comp.h == 0
    assert comp.const[2] == 1 and comp.const[3] == 1


def test_partial_zero_gate_rejected():
    """Zero entries that are neither diagonal nor a permutation (a
    controlled Hadamard) need the e^-J route, not exact elimination."""
    H = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    U = np.eye(4, dtype=complex)
    U[np.ix_([2, 3], [2, 3])] = H
    with pytest.raises(ocomp.CompileError):
        _one_gate(U, 2)


@pytest.mark.parametrize("name", ["tiny", "rct12", "brick20", "brick16"])
def test_workload_structure(name):
    """Gate sets {H, S, T, sqrt X, CNOT, CZ, CP}: every magnitude is
    constant, so the path law is uniform (one colour, no factors) and
    Z = 2^(h/2)."""
    comp = ocomp.compile_circuit(_circ(wc.workload_circuit(name)))
    assert comp.ncolours == 1
    assert all(len(f) == 0 for f in comp.factors)
    assert comp.Z == pytest.approx(2.0 ** (comp.h / 2), rel=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_magnitude_marginal_matches_enumeration(seed):
    """P_mag (magnitude circuit) equals the enumerated p_C marginal and
    Z = sum |psi_C| = product of column sums."""
    c = small_random(100 + seed)
    comp = ocomp.compile_circuit(c)
    pm, Z = exact.magnitude_marginal(c)
    marg = np.zeros(2 ** c.n)
    tot = 0.0
    amp = np.zeros(2 ** c.n, dtype=complex)
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        marg[a] += m
        tot += m
        amp[a] += m * cmath.exp(2j * math.pi * k / 2 ** c.K)
    assert tot == pytest.approx(Z, rel=1e-12)
    assert comp.Z == pytest.approx(Z, rel=1e-12)
    assert np.allclose(marg / tot, pm, atol=1e-12)
    # summing the compiled paths reproduces the statevector
    assert np.allclose(amp, exact.statevector(c), atol=1e-12)


def test_rotated_hadamard_theta():
    """Eq. (HadT): theta = pi/4 is the Hadamard gate (uniform law, one
    colour); theta = pi/2 is the classical NOT (no free p-bit)."""
    c = _circ(wc.rotated_hadamard_chain(6, math.pi / 4, K=1))
    comp = ocomp.compile_circuit(c)
    assert comp.h == 6 and all(not f for f in comp.factors)
    c2 = _circ(wc.rotated_hadamard_chain(6, math.pi / 2, K=1))
    comp2 = ocomp.compile_circuit(c2)
    assert comp2.h == 0
    c3 = _circ(wc.rotated_hadamard_chain(6, math.pi / 8, K=1))
    comp3 = ocomp.compile_circuit(c3)
    assert comp3.ncolours == 2 and comp3.h == 6
    # the path law is non-uniform and enumerates to the magnitude circuit
    pm, Z = exact.magnitude_marginal(c3)
    assert comp3.Z == pytest.approx(Z, rel=1e-12)


def test_nonsymmetric_gate_closed_form():
    """Gate orientation (rows = output, columns = input, Sec. 2): one H S
    gate maps |0> to its column 0, (1, 1)/sqrt(2), and |1> to column 1,
    (i, -i)/sqrt(2); S H maps |0> to (1, i)/sqrt(2).  Written out by hand."""
    r = 1.0 / math.sqrt(2.0)
    for kind, inp, want in [("HS", 0, [r, r]), ("HS", 1, [1j * r, -1j * r]), ("SH", 0, [r, 1j * r]),
                            ("SH", 1, [r, -1j * r])]:
        c = wc.circuit("one", 1, 1, 2, [wc.gate1(1, 0, kind)], inp)
        assert np.allclose(exact.statevector(_circ(c)), want, atol=1e-15), (kind, inp)
        assert np.allclose(exact.path_sum(_circ(c)), want, atol=1e-15), (kind, inp)


def compiled_amplitudes(comp):
    """Sum over the compiled lattice's paths of |psi_C| e^{2 pi i k / 2^K}
    per output state (Eq. (path) on the eliminated lattice)."""
    amp = np.zeros(2 ** comp.n, dtype=complex)
    for f, x, m, k, a in ocomp.enumerate_free(comp):
        amp[a] += m * cmath.exp(2j * math.pi * k / 2 ** comp.K)
    return amp


@pytest.mark.parametrize("seed", range(10))
def test_compiled_paths_reproduce_statevector(seed):
    """The compile (Appendix eliminations, magnitude and phase tables, cones)
    loses nothing: summing every path of the compiled lattice with its
    magnitude and phase bin gives the matrix-product amplitudes, for
    circuits with non-symmetric one-qubit gates (even seeds) and random
    Clifford+T circuits (odd seeds)."""
    c = small_asym(seed) if seed % 2 == 0 else small_random(seed)
    comp = ocomp.compile_circuit(c)
    assert np.allclose(compiled_amplitudes(comp), exact.statevector(c), atol=1e-12)


def test_repeated_cnot_cancels_in_the_lattice():
    """H(q0), CNOT(0->1), CNOT(0->1): the second CNOT undoes the first, so the
    state is (|0> + |1>)/sqrt(2) on qubit 0 with qubit 1 back to 0 (indices 0
    and 1, little-endian).  In the eliminated lattice qubit 1's last layer is
    x0 XOR x0 = 0; every path of the compiled lattice must reproduce it."""
    g = [wc.gate1(1, 0, "H"), wc.cnot(2, 0, 1), wc.cnot(3, 0, 1)]
    c = _circ(wc.circuit("cnot2", 2, 3, 1, g, 0))
    r = 1.0 / math.sqrt(2.0)
    want = np.array([r, r, 0, 0], dtype=complex)
    assert np.allclose(exact.statevector(c), want, atol=1e-15)
    comp = ocomp.compile_circuit(c)
    assert comp.h == 1
    assert np.allclose(compiled_amplitudes(comp), want, atol=1e-12)


@pytest.mark.parametrize("theta", [math.pi / 4, math.pi / 8, math.pi / 16, 3 * math.pi / 8, 0.3])
def test_prefactor_two_rotated_hadamards_closed_form(theta):
    """Eq. (U30) for d = 2 rotated Hadamards (Eq. (HadT)) worked by hand:
    to |0> the two paths weigh cos^2 and sin^2 (U = 1), so uniform sampling
    (p = 1/2, W = 2 psi) gives |cos 2 theta| and weighted sampling gives W = 1
    on both, std 0; to |1> they weigh +-sin cos (U = 0), both samplings give
    W = +-sin 2 theta, std |sin 2 theta|."""
    c = _circ(wc.rotated_hadamard_chain(2, theta, K=1))
    assert exact.prefactor(c, 0, False) == pytest.approx(abs(math.cos(2 * theta)), abs=1e-13)
    assert exact.prefactor(c, 0, True) == pytest.approx(0.0, abs=1e-7)
    assert exact.prefactor(c, 1, False) == pytest.approx(abs(math.sin(2 * theta)), abs=1e-13)
    assert exact.prefactor(c, 1, True) == pytest.approx(abs(math.sin(2 * theta)), abs=1e-13)


def test_prefactor_hadamard_chain_is_eq_stdT():
    """Fig. 5 at theta = pi/4 (the Hadamard gate): on the wrong output of
    d = 10 the prefactor is the 2^(d/2) / 2 of Eq. (stdT) (std(T) times the
    root of the T/2 samples that reach it), and weighted sampling equals
    uniform sampling on both outputs (all paths weigh the same)."""
    c = _circ(wc.rotated_hadamard_chain(10, math.pi / 4, K=1))
    assert exact.prefactor(c, 1, False) == pytest.approx(2.0 ** 5 / 2, rel=1e-12)
    for a in (0, 1):
        assert exact.prefactor(c, a, True) == pytest.approx(exact.prefactor(c, a, False), rel=1e-12)


@pytest.mark.parametrize("theta", [math.pi / 32, math.pi / 8, 0.5, math.pi / 3, 0.45 * math.pi])
def test_prefactor_weighted_closed_form_and_ordering(theta):
    """Weighted sampling (p_C = |psi_C| / Z_alpha over the paths to alpha)
    makes W_C = Z_alpha times a phase, so Eq. (U30) is sqrt(Z_alpha^2 -
    |U_alpha|^2): checked against Z_alpha from the magnitude circuit and
    U_alpha from the statevector (independent routines).  By Cauchy-Schwarz
    it never exceeds uniform sampling (Fig. 5's point), and at theta = pi/2
    (a classical NOT) it is zero."""
    c = _circ(wc.rotated_hadamard_chain(10, theta, K=1))
    pm, Z = exact.magnitude_marginal(c)
    psi = exact.statevector(c)
    for a in (0, 1):
        Za = pm[a] * Z
        want = math.sqrt(max(Za * Za - abs(psi[a]) ** 2, 0.0))
        assert exact.prefactor(c, a, True) == pytest.approx(want, rel=1e-9, abs=1e-12)
        assert exact.prefactor(c, a, True) <= exact.prefactor(c, a, False) + 1e-12
    cx = _circ(wc.rotated_hadamard_chain(10, math.pi / 2, K=1))
    assert exact.prefactor(cx, 0, True) == pytest.approx(0.0, abs=1e-12)
    assert exact.prefactor(cx, 0, False) > 1.0
