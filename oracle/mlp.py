"""FP64 oracle for the learned SCF mixer (the preconditioner network of the
self-consistent response loop).  TEST INFRASTRUCTURE ONLY (see
oracle/__init__.py).

The network is applied site by site with shared weights: for a residual
vector x in R^n (one self-consistent state) the input of site i is
    z_i = [x_{i-w}, ..., x_{i+w}, e_{i-w}, ..., e_{i+w}, U_i]
                          (k = 4w + 3 features; x_j = e_j = 0 outside 0..n-1),
with e the on-site energies (diagonal of H0), which tell the network where
the polarisable sites are.
and the output is the scalar
    y_i = w2 . tanh(W1 z_i + b1) + b2,
a two-layer network of hidden width h.  Parameters are one vector
[W1 (h x k, row-major), b1 (h), w2 (h), b2 (1)].  Loss over a batch of B
states: the mean squared error L = (1 / (B n)) sum_{b,i} (y_bi - t_bi)^2.
Training uses Adam (Kingma & Ba, 2015): m = b1 m + (1 - b1) g,
v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def features(window: int) -> int:
    return 4 * window + 3


def param_count(window: int, h: int) -> int:
    k = features(window)
    return h * k + h + h + 1


def unpack(p: np.ndarray, window: int, h: int):
    p = np.asarray(p, np.float64)
    k = features(window)
    o = 0
    w1 = p[o:o + h * k].reshape(h, k); o += h * k
    b1 = p[o:o + h]; o += h
    w2 = p[o:o + h]; o += h
    b2 = p[o]
    return w1, b1, w2, b2


def site_inputs(x: np.ndarray, u: np.ndarray, e: np.ndarray, window: int) -> np.ndarray:
    """(B, n) states -> (B * n, k) site inputs, rows ordered (b, i)."""
    x = np.asarray(x, np.float64)
    e = np.asarray(e, np.float64)
    bsz, n = x.shape
    k = features(window)
    m = 2 * window + 1
    z = np.zeros((bsz, n, k))
    for d in range(-window, window + 1):
        lo, hi = max(0, -d), min(n, n - d)          # sites i with 0 <= i + d < n
        if lo < hi:                                 # none when |d| >= n
            z[:, lo:hi, d + window] = x[:, lo + d:hi + d]
            z[:, lo:hi, m + d + window] = e[None, lo + d:hi + d]
    z[:, :, k - 1] = np.asarray(u, np.float64)[None, :]
    return z.reshape(bsz * n, k)


def forward(p, x, u, e, window: int, h: int):
    """x: (B, n) -> (y (B, n), site inputs, hidden activations)."""
    w1, b1, w2, b2 = unpack(p, window, h)
    bsz, n = np.asarray(x).shape
    z = site_inputs(x, u, e, window)
    a = np.tanh(z @ w1.T + b1)
    return (a @ w2 + b2).reshape(bsz, n), z, a


def loss_grad(p, x, t, u, e, window: int, h: int):
    """(loss, gradient with respect to the packed parameters)."""
    w1, b1, w2, b2 = unpack(p, window, h)
    y, z, a = forward(p, x, u, e, window, h)
    r = (y - np.asarray(t, np.float64)).ravel()
    m = r.size
    loss = float(r @ r / m)
    dy = 2.0 * r / m
    gw2 = a.T @ dy
    gb2 = dy.sum()
    dz = np.outer(dy, w2) * (1.0 - a * a)
    gw1 = dz.T @ z
    gb1 = dz.sum(axis=0)
    return loss, np.concatenate([gw1.ravel(), gb1, gw2, [gb2]])


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step counts from 1); returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
