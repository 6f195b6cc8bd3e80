"""Period finding by column sampling (Sec. 5, Fig. 7) (test infrastructure only).

The first register has n p-bits; a sample is a configuration x of it, drawn
uniformly (the bank of Hadamards gives every x the same weight).  Its
second-register value is f(x) = a^x mod N (the modular exponentiation, a
deterministic map).  The inverse QFT maps |x> to 2^(-n/2) sum_k
exp(-2 pi i k x / 2^n) |k>: that column is added to column f(x) of psi
(2^n rows k, one column per value of f), and the output probabilities are
the row sums of |psi|^2.  With T samples and the normalisation used here

    P[k] = 2^(-n) / T * sum over values f of |sum over sampled x with
           f(x) = f of exp(-2 pi i k x / 2^n)|^2,

so that P sums to 1 when no x is drawn twice.  Plain and slow, FP64.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

from . import chain

TAG_SHOR = 3


def draws(n, T, seed):
    """x_i = low n bits of word i mod 4 of Philox4x32-10 at counter
    (i // 4, 0, 0, 3 << 16) under key (seed lo, seed hi): uniform over 2^n."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    mask = (1 << n) - 1
    out = []
    for i in range(T):
        if i % 4 == 0:
            block = chain.philox((i // 4, 0, 0, TAG_SHOR << 16), key)
        out.append(block[i % 4] & mask)
    return out


def groups(N, a, xs):
    """The sampled x grouped by f(x) = a^x mod N: {f: [x, ...]}."""
    g = {}
    for x in xs:
        g.setdefault(pow(a, x, N), []).append(x)
    return g


def column_probs(N, a, n, xs, ks=None):
    """P[k] above, for k in ks (default all 2^n)."""
    ks = range(2 ** n) if ks is None else ks
    g = groups(N, a, xs)
    T = len(xs)
    out = []
    for k in ks:
        tot = 0.0
        for members in g.values():
            s = sum(cmath.exp(-2j * math.pi * ((k * x) % 2 ** n) / 2 ** n) for x in members)
            tot += abs(s) ** 2
        out.append(tot / (2 ** n * T))
    return np.array(out)


def register_distribution(N, a, n):
    """The output law of the first register from the circuit of Fig. 6 with
    t = n qubits, built as matrices: |0...0>|1> -> Hadamards -> |x>|a^x mod
    N> -> inverse QFT on the first register -> P[k] = sum_y |amp[k, y]|^2
    (tiny n only).  The column-sampling P with every x drawn once equals it."""
    dim = 2 ** n
    psi = np.zeros((dim, N), dtype=np.complex128)
    for x in range(dim):
        psi[x, pow(a, x, N)] = dim ** -0.5
    kk, xx = np.meshgrid(np.arange(dim), np.arange(dim), indexing="ij")
    F = np.exp(-2j * np.pi * kk * xx / dim) / math.sqrt(dim)
    out = F @ psi
    return (np.abs(out) ** 2).sum(axis=1)


def order(N, a):
    """Multiplicative order r of a mod N (brute force)."""
    v, r = a % N, 1
    while v != 1:
        v = v * a % N
        r += 1
        if r > N:
            raise ValueError("a is not invertible mod N")
    return r
