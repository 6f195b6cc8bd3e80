"""Pins of the oracle MADE to mathematics other than itself: finite
differences, the autoregressive property, normalisation over all inputs,
and Adam's closed form for a constant gradient."""
import itertools

import numpy as np
import pytest

from oracle import made


def _params(D, H, seed):
    rng = np.random.default_rng(seed)
    M1, M2, M3 = made.masks(D, H)
    W1 = rng.normal(0, 0.7, (D, H)) * M1
    W2 = rng.normal(0, 0.4, (H, H)) * M2
    V = rng.normal(0, 0.4, (H, D)) * M3
    b1 = rng.normal(0, 0.3, H)
    b2 = rng.normal(0, 0.3, H)
    c = rng.normal(0, 0.3, D)
    return [W1, b1, W2, b2, V, c]


def test_gradients_match_central_differences():
    D, H = 8, 16
    p = _params(D, H, 0)
    rng = np.random.default_rng(1)
    X = rng.integers(0, 2, (5, D)).astype(float)
    free = np.array([1, 1, 0, 1, 1, 0, 1, 1], dtype=bool)
    _, grads = made.loss_and_grads(p, X, free)
    masks = made.masks(D, H)
    mask_of = {0: masks[0], 2: masks[1], 4: masks[2]}
    eps = 1e-6
    for pi in range(6):
        g = grads[pi]
        it = np.nditer(p[pi], flags=["multi_index"])
        checked = 0
        for _ in it:
            idx = it.multi_index
            if pi in mask_of and mask_of[pi][idx] == 0:
                assert g[idx] == 0.0
                continue
            if checked > 25:
                break
            old = p[pi][idx]
            p[pi][idx] = old + eps
            lp, _ = made.loss_and_grads(p, X, free)
            p[pi][idx] = old - eps
            lm, _ = made.loss_and_grads(p, X, free)
            p[pi][idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[idx]) < 1e-6 * max(1.0, abs(fd)), (pi, idx, fd, g[idx])
            checked += 1


def test_autoregressive_property():
    """Logit o never depends on inputs at positions >= o."""
    D, H = 10, 24
    p = _params(D, H, 2)
    rng = np.random.default_rng(3)
    x = rng.integers(0, 2, (1, D)).astype(float)
    L0, _ = made.forward(p, x)
    for i in range(D):
        x2 = x.copy()
        x2[0, i] = 1 - x2[0, i]
        L1, _ = made.forward(p, x2)
        changed = np.abs(L1 - L0)[0] > 0
        assert not changed[: i + 1].any(), i


def test_log_q_normalises():
    D, H = 7, 12
    p = _params(D, H, 4)
    X = np.array(list(itertools.product([0, 1], repeat=D)), dtype=float)
    free = np.ones(D, dtype=bool)
    q = np.exp(made.log_q(p, X, free))
    assert q.sum() == pytest.approx(1.0, rel=1e-12)


def test_adam_constant_gradient_closed_form():
    theta = np.array([0.5, -1.0, 2.0])
    g = np.array([0.3, -2.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    lr, eps = 1e-3, 1e-8
    th = theta.copy()
    for t in range(1, 21):
        th, m, v = made.adam_step(th, m, v, g, t, lr=lr, eps=eps)
    # constant g: bias-corrected m = g, v = g^2 at every step
    want = theta - 20 * lr * g / (np.abs(g) + eps)
    assert np.allclose(th, want, rtol=1e-12, atol=1e-15)


def test_each_output_sees_its_predecessor():
    """The masks keep every allowed connection: with generic weights logit o
    changes when input o - 1 flips (a mask one degree too strict would cut
    it)."""
    D, H = 10, 40
    p = _params(D, H, 5)
    rng = np.random.default_rng(6)
    x = rng.integers(0, 2, (1, D)).astype(float)
    L0, _ = made.forward(p, x)
    for o in range(1, D):
        x2 = x.copy()
        x2[0, o - 1] = 1 - x2[0, o - 1]
        L1, _ = made.forward(p, x2)
        assert abs(L1[0, o] - L0[0, o]) > 1e-9, o
