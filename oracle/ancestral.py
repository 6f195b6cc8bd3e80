"""An independent exact sampler of the path law of Eq. (weightedS)
(test infrastructure only).

Paths are drawn forward, layer by layer: at each gate the output state is
drawn with probability |U[out][in]| / c_g(in), c_g(in) = sum_out |U[out][in]|.
The probability of a whole path is then prod_g |U_g| / c_g, which equals
|psi_C| / Z when every c_g is constant over its inputs (every unitary
one-qubit gate and every permutation-type gate has that property), so the
draws are iid from p_C.  Used only to cross-check the Gibbs replay.
"""
from __future__ import annotations

import math

import numpy as np


def sample(circ, T, seed, K=None):
    """Draw T iid paths; returns counts[2^n, 2^K] of (alpha, phase bin)."""
    K = circ.K if K is None else K
    rng = np.random.default_rng(seed)
    n = circ.n
    state = np.full(T, circ.input, dtype=np.int64)
    phase = np.zeros(T, dtype=np.int64)
    step = 2.0 * math.pi / (2 ** K)
    for g in circ.gates:
        dim = 2 ** g.arity
        mag = np.abs(g.U)
        cols = mag.sum(axis=0)
        if cols.max() - cols.min() > 1e-9 * cols.max():
            raise ValueError("column sums not constant: ancestral sampling is not exact")
        sub = np.zeros(T, dtype=np.int64)
        for j, q in enumerate(g.qubits):
            sub |= ((state >> q) & 1) << j
        u = rng.random(T)
        cdf = np.cumsum(mag / cols[None, :], axis=0)     # [out, in]
        out = np.zeros(T, dtype=np.int64)
        for o in range(dim - 1):
            out += (u >= cdf[o, sub]).astype(np.int64)
        ang = np.angle(g.U[out, sub])
        phase += np.rint(ang / step).astype(np.int64)
        for j, q in enumerate(g.qubits):
            state &= ~(1 << q)
            state |= ((out >> j) & 1) << q
    phase %= 2 ** K
    counts = np.zeros((2 ** n, 2 ** K), dtype=np.int64)
    np.add.at(counts, (state, phase), 1)
    return counts
