"""Exact results the sampler must reproduce (test infrastructure only).

* `statevector` -- U_{alpha,beta} for all alpha as the matrix product of
  Eq. (U): the gates are applied one by one to the basis state beta.
* `path_sum` -- the same amplitudes as the explicit sum over every Feynman
  path of Eq. (path): every lattice configuration beta -> p_1 -> ... -> alpha
  is enumerated and its product of gate entries added to its output bin.
  Idle qubits carry the identity, so a path that changes an idle qubit has
  weight zero.
* `magnitude_marginal` -- the output marginal of the sampling law of
  Eq. (weightedS), p_C proportional to |prod U|, obtained by running the
  circuit with every gate matrix replaced by its entrywise modulus; its
  total is Z = sum_C |psi_C|.

Everything is FP64.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _apply(psi, n, qubits, U):
    """Apply the 2^a x 2^a matrix U (rows = output, index s_{q0}+2 s_{q1})
    to the n-qubit tensor psi, whose numpy axis for qubit q is n-1-q."""
    a = len(qubits)
    Ut = U.reshape([2] * (2 * a))          # axes: o_{a-1}..o_0, i_{a-1}..i_0
    in_axes = [n - 1 - q for q in reversed(qubits)]   # i_{a-1} .. i_0
    out = np.tensordot(Ut, psi, axes=(list(range(a, 2 * a)), in_axes))
    # out axes: o_{a-1}..o_0, then psi's remaining axes in order
    return np.moveaxis(out, list(range(a)), in_axes)


def _run(circ, mats, dtype):
    n = circ.n
    psi = np.zeros(2 ** n, dtype=dtype)
    psi[circ.input] = 1.0
    psi = psi.reshape([2] * n)
    for g, U in zip(circ.gates, mats):
        psi = _apply(psi, n, g.qubits, U)
    return psi.reshape(2 ** n)


def statevector(circ):
    """Column beta of U^(d) ... U^(1), Eq. (U)."""
    return _run(circ, [g.U for g in circ.gates], np.complex128)


def magnitude_marginal(circ):
    """(P_mag, Z): P_mag[alpha] = sum over paths ending in alpha of
    |psi_C| / Z with Z = sum over all paths of |psi_C| (Eq. (weightedS))."""
    v = _run(circ, [np.abs(g.U) for g in circ.gates], np.float64)
    Z = float(v.sum())
    return v / Z, Z


def dense_unitary(circ):
    """Full 2^n x 2^n product of layer matrices, built from Kronecker
    products (tiny n only); an independent route to Eq. (U)."""
    n = circ.n
    dim = 2 ** n
    total = np.eye(dim, dtype=np.complex128)
    for layer in range(1, circ.d + 1):
        M = np.eye(dim, dtype=np.complex128)
        for g in [g for g in circ.gates if g.layer == layer]:
            G = np.zeros((dim, dim), dtype=np.complex128)
            for col in range(dim):
                sub_in = sum(((col >> q) & 1) << j for j, q in enumerate(g.qubits))
                base = col
                for q in g.qubits:
                    base &= ~(1 << q)
                for o in range(2 ** g.arity):
                    row = base
                    for j, q in enumerate(g.qubits):
                        row |= ((o >> j) & 1) << q
                    G[row, col] += g.U[o, sub_in]
            M = G @ M
        total = M @ total
    return total


def path_sum(circ, return_paths=False):
    """Explicit Feynman-path sum of Eq. (path) over all 2^(n d) lattice
    configurations whose layer 0 equals the input state.  Returns the
    amplitude vector over alpha (and, optionally, the list of nonzero paths
    as (layers tuple, psi_C))."""
    n, d = circ.n, circ.d
    by_layer = {l: [] for l in range(1, d + 1)}
    for g in circ.gates:
        by_layer[g.layer].append(g)
    amp = np.zeros(2 ** n, dtype=np.complex128)
    paths = []
    for mid in itertools.product(range(2 ** n), repeat=d):
        states = (circ.input,) + mid
        w = 1.0 + 0.0j
        for l in range(1, d + 1):
            prev, cur = states[l - 1], states[l]
            touched = 0
            for g in by_layer[l]:
                i = sum(((prev >> q) & 1) << j for j, q in enumerate(g.qubits))
                o = sum(((cur >> q) & 1) << j for j, q in enumerate(g.qubits))
                w *= g.U[o, i]
                for q in g.qubits:
                    touched |= 1 << q
            idle = ((1 << n) - 1) & ~touched
            if (prev ^ cur) & idle:
                w = 0.0
            if w == 0:
                break
        if w != 0:
            amp[states[-1]] += w
            if return_paths:
                paths.append((states, w))
    if return_paths:
        return amp, paths
    return amp


def prefactor(circ, alpha, weighted):
    """std({W_C},{p_C}) of Eq. (U30) over the paths of Eq. (U343) that end
    in output alpha, the quantity Fig. 5 plots for a chain of rotated
    Hadamards: W_C = psi_C / p_C (Eq. (U344)) and U = sum of psi_C over those
    paths; p_C is uniform over all 2^(n(d-1)) intermediate sequences ending
    in alpha (weighted=False; paths of weight zero included) or
    proportional to |psi_C| among them (weighted=True, Eq. (weightedS)).
    |W - U|^2 is used for complex weights.  Explicit enumeration: tiny
    circuits only."""
    _, paths = path_sum(circ, return_paths=True)
    mine = [w for states, w in paths if states[-1] == alpha]
    U = complex(sum(mine))
    if weighted:
        Za = float(sum(abs(w) for w in mine))
        if Za == 0.0:
            return 0.0
        var = sum((abs(w) / Za) * abs(w / (abs(w) / Za) - U) ** 2 for w in mine)
    else:
        N = 2 ** (circ.n * (circ.d - 1))
        var = sum((1.0 / N) * abs(w * N - U) ** 2 for w in mine)
        var += (N - len(mine)) * (1.0 / N) * abs(U) ** 2  # the paths of weight zero
    return math.sqrt(max(var, 0.0))
