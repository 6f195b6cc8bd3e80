"""FP64 MADE (masked autoencoder for distribution estimation; Germain,
Gregor, Murray, Larochelle, ICML 2015) -- test infrastructure only.

The learned proposal is not part of the paper (its Boltzmann machine is not
trained, Sec. 1); it is an independence proposal inside the Metropolis-
Hastings accept of Fig. 2 step 2.  The network is plain and written out here
in float64 so that the GPU's forward, backward and Adam can be checked:

  degrees: input position i (0-based) has degree i + 1; hidden unit k of a
           layer of width H over D positions has degree
           1 + floor(k (D - 1) / H) (ascending, values 1..D-1);
  masks:   a weight from a unit of degree a to a unit of degree b is allowed
           iff a <= b, with output position o given degree o (so its logit
           only sees hidden units of degree <= o, i.e. inputs < o);
  network: H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), L = H2 V + c;
  loss:    mean over the batch of the binary cross-entropy summed over the
           free positions (deterministic positions carry no loss);
  Adam:    m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
           theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def hidden_degrees(D, H):
    k = np.arange(H)
    return 1 + (k * (D - 1)) // H


def masks(D, H):
    din = np.arange(1, D + 1)
    d1 = hidden_degrees(D, H)
    d2 = hidden_degrees(D, H)
    dout = np.arange(D)
    M1 = (din[:, None] <= d1[None, :]).astype(np.float64)     # [D, H]
    M2 = (d1[:, None] <= d2[None, :]).astype(np.float64)      # [H, H]
    M3 = (d2[:, None] <= dout[None, :]).astype(np.float64)    # [H, D]
    return M1, M2, M3


def forward(params, X):
    W1, b1, W2, b2, V, c = params
    A1 = X @ W1 + b1
    H1 = np.maximum(A1, 0.0)
    A2 = H1 @ W2 + b2
    H2 = np.maximum(A2, 0.0)
    L = H2 @ V + c
    return L, (X, A1, H1, A2, H2)


def _log_sigmoid(z):
    return -np.logaddexp(0.0, -z)


def loss_and_grads(params, X, free_mask):
    """Mean over the batch of sum over free positions of BCE; gradients of
    every parameter (the masks are applied by the caller's parametrisation:
    gradients are multiplied by the masks here)."""
    W1, b1, W2, b2, V, c = params
    B, D = X.shape
    M1, M2, M3 = masks(D, W1.shape[1])
    L, (X_, A1, H1, A2, H2) = forward(params, X)
    f = free_mask[None, :].astype(np.float64)
    nll = -(X * _log_sigmoid(L) + (1 - X) * _log_sigmoid(-L)) * f
    loss = nll.sum() / B
    sig = 1.0 / (1.0 + np.exp(-L))
    G3 = (sig - X) * f / B                     # dloss/dL
    dV = H2.T @ G3 * M3
    dc = G3.sum(axis=0)
    G2 = (G3 @ V.T) * (A2 > 0)
    dW2 = H1.T @ G2 * M2
    db2 = G2.sum(axis=0)
    G1 = (G2 @ W2.T) * (A1 > 0)
    dW1 = X.T @ G1 * M1
    db1 = G1.sum(axis=0)
    return loss, (dW1, db1, dW2, db2, dV, dc)


def adam_step(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def log_q(params, X, free_mask):
    """log q(x) = sum over free positions of log q(x_i | x_<i)."""
    L, _ = forward(params, X)
    f = free_mask[None, :].astype(np.float64)
    return ((X * _log_sigmoid(L) + (1 - X) * _log_sigmoid(-L)) * f).sum(axis=1)
