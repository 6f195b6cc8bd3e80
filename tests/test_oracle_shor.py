"""Pins of the column-sampling oracle (Sec. 5, Figs. 6-7) against the
circuit built as matrices, closed forms and identities."""
import math

import numpy as np
import pytest

from oracle import shor


def test_n15_a7_closed_form():
    """a = 7 has order 4 mod 15 and 4 divides 2^4: the inverse QFT leaves
    mass 1/4 on k = 0, 4, 8, 12 and nothing elsewhere (written out by hand)."""
    P = shor.register_distribution(15, 7, 4)
    want = np.zeros(16)
    want[[0, 4, 8, 12]] = 0.25
    assert np.allclose(P, want, atol=1e-14)


@pytest.mark.parametrize("N,a,n", [(15, 7, 4), (21, 2, 5), (35, 3, 6), (15, 2, 5), (33, 5, 6)])
def test_all_columns_once_equals_circuit(N, a, n):
    """Every x drawn exactly once: the column-sampling P equals the output
    law of the circuit of Fig. 6 with t = n (built from matrices)."""
    P = shor.column_probs(N, a, n, list(range(2 ** n)))
    assert np.allclose(P, shor.register_distribution(N, a, n), atol=1e-12)
    assert P.sum() == pytest.approx(1.0, abs=1e-12)


def test_peaks_at_multiples_of_2n_over_r():
    """Order 6 mod 21 does not divide 2^5: the six largest probabilities sit
    at the integers nearest j 2^n / r, j = 0..r-1."""
    N, a, n = 21, 2, 5
    r = shor.order(N, a)
    assert r == 6
    P = shor.register_distribution(N, a, n)
    top = set(np.argsort(P)[::-1][:r].tolist())
    assert top == {int(round(j * 2 ** n / r)) % 2 ** n for j in range(r)}


def test_sampled_identities():
    """Sampled x: P is symmetric under k -> 2^n - k, sums to sum_x m_x^2 / T
    (m_x = times x was drawn; Parseval), and the draws lie below 2^n."""
    N, a, n, T = 35, 3, 6, 50
    xs = shor.draws(n, T, 99)
    assert all(0 <= x < 2 ** n for x in xs)
    P = shor.column_probs(N, a, n, xs)
    assert np.allclose(P[1:], P[1:][::-1], atol=1e-13)
    m = np.bincount(xs, minlength=2 ** n)
    assert P.sum() == pytest.approx(float((m * m).sum()) / T, rel=1e-12)


def test_order():
    for N, a in [(15, 7), (21, 2), (98743069, 10424)]:
        r = shor.order(N, a)
        assert pow(a, r, N) == 1
        assert all(pow(a, d, N) != 1 for d in range(1, r) if r % d == 0)
    assert shor.order(98743069, 10424) == 78  # Fig. 8's period
