"""Planted mistakes: each test plants one plausible error in the oracle (on
the CPU, for the duration of the test only) and checks that at least one of
the oracle's pins fails, so the pins would have caught it."""
import math

import numpy as np
import pytest

from oracle import compile as ocomp
from oracle import estimator as oest
from oracle import exact
from oracle import made as omade
from oracle import shor as oshor

import test_oracle_chain as tchain  # tests/ is on sys.path under pytest
import test_oracle_estimator as testim
import test_oracle_exact as texact
import test_oracle_made as tmade
import test_oracle_shor as tshor
import test_oracle_nonlinear as tnl


def caught(*pins):
    """True if at least one pin (callable, or (callable, args)) fails."""
    for pin in pins:
        fn, args = (pin, ()) if callable(pin) else pin
        try:
            fn(*args)
        except AssertionError:
            return True
    return False


EXACT_PINS = [texact.test_nonsymmetric_gate_closed_form, texact.test_tiny_amplitudes_and_phase_bins,
              texact.test_hadamard_d2_worked_example, texact.test_repeated_cnot_cancels_in_the_lattice] + [
    (texact.test_statevector_equals_path_sum_and_dense, (s,)) for s in range(18)] + [
    (texact.test_compiled_paths_reproduce_statevector, (s,)) for s in range(10)]


def test_transposed_gate_matrix_is_caught(monkeypatch):
    orig = exact._apply
    monkeypatch.setattr(exact, "_apply", lambda psi, n, qubits, U: orig(psi, n, qubits, U.T))
    assert caught(*EXACT_PINS)


def test_conjugated_gate_matrix_is_caught(monkeypatch):
    orig = exact._apply
    monkeypatch.setattr(exact, "_apply", lambda psi, n, qubits, U: orig(psi, n, qubits, U.conj()))
    assert caught(*EXACT_PINS)


class _NegAtan2:
    """math with atan2 negated: every phase bin gets the wrong sign."""

    def __getattr__(self, name):
        if name == "atan2":
            return lambda y, x: -math.atan2(y, x)
        return getattr(math, name)


def test_phase_sign_flip_in_compile_is_caught(monkeypatch):
    monkeypatch.setattr(ocomp, "math", _NegAtan2())
    assert caught(*EXACT_PINS)


def test_swapped_table_index_in_compile_is_caught(monkeypatch):
    def index(self, bits):
        i = sum(int(bits[p]) << j for j, p in enumerate(self.in_bits))
        o = sum(int(bits[p]) << j for j, p in enumerate(self.out_bits))
        return i * (2 ** self.a) + o  # rows and columns exchanged
    monkeypatch.setattr(ocomp.OGate, "index", index)
    assert caught(*EXACT_PINS)


def test_or_instead_of_xor_in_cones_is_caught(monkeypatch):
    monkeypatch.setattr(ocomp, "_xor", lambda f1, f2: (f1[0] | f2[0], f1[1] | f2[1]))
    assert caught(*EXACT_PINS)


def test_dropped_path_in_path_sum_is_caught(monkeypatch):
    orig = exact.path_sum

    def path_sum(circ, return_paths=False):
        amp, paths = orig(circ, return_paths=True)
        if paths:
            s, w = paths[-1]
            amp = amp.copy()
            amp[s[-1] if isinstance(s[-1], (int, np.integer)) else 0] -= w
            paths = paths[:-1]
        return (amp, paths) if return_paths else amp
    monkeypatch.setattr(exact, "path_sum", path_sum)
    assert caught(*EXACT_PINS)


CHAIN_PINS = [tchain.test_tiny_chain_support_and_amplitudes]


def test_conjugated_phase_in_estimator_is_caught(monkeypatch):
    orig = oest._omega
    monkeypatch.setattr(oest, "_omega", lambda K: (orig(K)[0], -orig(K)[1]))
    assert caught(*CHAIN_PINS)


def test_missing_normalisation_in_estimator_is_caught(monkeypatch):
    orig = oest.amplitudes
    monkeypatch.setattr(oest, "amplitudes", lambda counts, Z, T=None: orig(counts, 1.0, T))
    assert caught(*CHAIN_PINS)


def test_sigma_without_factor_two_in_denominator_is_caught(monkeypatch):
    orig = oest.exact_sigma

    def exact_sigma(prob, Z, T):
        sre, sim = orig(prob, Z, T)
        return sre * math.sqrt(2.0), sim
    monkeypatch.setattr(oest, "exact_sigma", exact_sigma)
    assert caught((texact.test_sigma_wrong_output_eq_stdT, (4,)), texact.test_tiny_sigma_closed_form)


ESTIMATOR_PINS = [testim.test_tiny_at_expectation_exact_z_and_l2_give_psi,
                  testim.test_l2_mode_is_scale_free_and_unit_norm] + [
    (testim.test_hadamard_chain_at_expectation, (d,)) for d in (2, 4, 8)] + [
    (testim.test_random_circuits_at_expectation_match_statevector, (s,)) for s in range(4)]


def test_l1_norm_in_l2_mode_is_caught(monkeypatch):
    """Fig. 2 step 4 normalises by the L2 norm; an L1 norm is a plausible slip."""
    def amplitudes_l2(counts):
        counts = np.asarray(counts, dtype=np.float64)
        K = int(round(math.log2(counts.shape[1])))
        cs, sn = oest._omega(K)
        A = counts @ cs + 1j * (counts @ sn)
        nrm = float(np.sum(np.abs(A)))
        return A / nrm if nrm > 0 else A
    monkeypatch.setattr(oest, "amplitudes_l2", amplitudes_l2)
    assert caught(*ESTIMATOR_PINS)


def test_missing_square_root_in_l2_mode_is_caught(monkeypatch):
    def amplitudes_l2(counts):
        counts = np.asarray(counts, dtype=np.float64)
        K = int(round(math.log2(counts.shape[1])))
        cs, sn = oest._omega(K)
        A = counts @ cs + 1j * (counts @ sn)
        nrm = float(np.sum(np.abs(A) ** 2))
        return A / nrm if nrm > 0 else A
    monkeypatch.setattr(oest, "amplitudes_l2", amplitudes_l2)
    assert caught(*ESTIMATOR_PINS)


def test_sigma_off_by_root_two_in_count_estimator_is_caught(monkeypatch):
    """The sigma computed from counts (Eq. (U26)), not only exact_sigma."""
    orig = oest.amplitudes

    def amplitudes(counts, Z, T=None):
        amp, sre, sim = orig(counts, Z, T)
        return amp, sre / math.sqrt(2.0), sim / math.sqrt(2.0)
    monkeypatch.setattr(oest, "amplitudes", amplitudes)
    assert caught(*ESTIMATOR_PINS)


def test_sigma_without_mean_subtraction_is_caught(monkeypatch):
    """Var = E W^2 - (E W)^2; dropping the square of the mean."""
    def amplitudes(counts, Z, T=None):
        counts = np.asarray(counts, dtype=np.float64)
        K = int(round(math.log2(counts.shape[1])))
        T = float(counts.sum()) if T is None else float(T)
        cs, sn = oest._omega(K)
        f = counts / T
        amp = Z * (f @ cs + 1j * (f @ sn))
        return amp, np.sqrt(Z * Z * (f @ (cs * cs)) / T), np.sqrt(Z * Z * (f @ (sn * sn)) / T)
    monkeypatch.setattr(oest, "amplitudes", amplitudes)
    assert caught(*ESTIMATOR_PINS)


MADE_PINS = [tmade.test_gradients_match_central_differences, tmade.test_autoregressive_property,
             tmade.test_log_q_normalises, tmade.test_adam_constant_gradient_closed_form,
             tmade.test_each_output_sees_its_predecessor]


def test_too_strict_first_mask_is_caught(monkeypatch):
    orig = omade.masks

    def masks(D, H):
        M1, M2, M3 = orig(D, H)
        din = np.arange(1, D + 1)
        d1 = omade.hidden_degrees(D, H)
        return (din[:, None] < d1[None, :]).astype(np.float64), M2, M3
    monkeypatch.setattr(omade, "masks", masks)
    assert caught(*MADE_PINS)


def test_too_loose_output_mask_is_caught(monkeypatch):
    orig = omade.masks

    def masks(D, H):
        M1, M2, M3 = orig(D, H)
        d2 = omade.hidden_degrees(D, H)
        dout = np.arange(D)
        return M1, M2, (d2[:, None] <= dout[None, :] + 1).astype(np.float64)
    monkeypatch.setattr(omade, "masks", masks)
    assert caught(*MADE_PINS)


def test_adam_without_bias_correction_is_caught(monkeypatch):
    def adam_step(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        return theta - lr * m / (np.sqrt(v) + eps), m, v
    monkeypatch.setattr(omade, "adam_step", adam_step)
    assert caught(*MADE_PINS)


def test_wrong_sign_in_loss_gradient_is_caught(monkeypatch):
    orig = omade.loss_and_grads

    def loss_and_grads(params, X, free_mask):
        loss, g = orig(params, X, free_mask)
        return loss, tuple(-x if i == 4 else x for i, x in enumerate(g))
    monkeypatch.setattr(omade, "loss_and_grads", loss_and_grads)
    assert caught(*MADE_PINS)


NONLINEAR_PINS = [tnl.test_toffoli_truth_table] + [
    (tnl.test_compiled_paths_with_toffoli_reproduce_statevector, (s,)) for s in range(8)]


def test_inverted_permutation_in_forward_lattice_is_caught(monkeypatch):
    orig = ocomp.forward_lattice

    def forward_lattice(comp, f):
        saved = [(g, g.perm) for g in comp.gates if g.perm is not None]
        try:
            for g, p in saved:
                g.perm = [p.index(i) for i in range(len(p))]
            return orig(comp, f)
        finally:
            for g, p in saved:
                g.perm = p
    monkeypatch.setattr(ocomp, "forward_lattice", forward_lattice)
    assert caught(*NONLINEAR_PINS)


SHOR_PINS = [tshor.test_n15_a7_closed_form, tshor.test_peaks_at_multiples_of_2n_over_r] + [
    (tshor.test_all_columns_once_equals_circuit, args) for args in [(15, 7, 4), (21, 2, 5)]]


def test_columns_grouped_by_x_instead_of_f_is_caught(monkeypatch):
    monkeypatch.setattr(oshor, "groups", lambda N, a, xs: {x: [x] for x in xs})
    assert caught(*SHOR_PINS)


def test_inverse_qft_without_normalisation_is_caught(monkeypatch):
    orig = oshor.register_distribution
    monkeypatch.setattr(oshor, "register_distribution", lambda N, a, n: orig(N, a, n) * 2 ** n)
    assert caught(*SHOR_PINS)


@pytest.mark.parametrize("pin", EXACT_PINS[:4] + CHAIN_PINS + ESTIMATOR_PINS + MADE_PINS + SHOR_PINS
                         + NONLINEAR_PINS[:2],
                         ids=lambda p: getattr(p, "__name__", str(p)))
def test_pins_pass_on_the_unmodified_oracle(pin):
    """Control: the same pins pass when nothing is planted."""
    assert not caught(pin)
