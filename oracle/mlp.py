"""FP64 oracle for the learned SCF mixer (the preconditioner network of the
self-consistent response loop).  TEST INFRASTRUCTURE ONLY (see
oracle/__init__.py).

Network: x in R^n -> y = W2 tanh(W1 x + b1) + b2 in R^n, hidden width h.
Parameters are one vector [W1 (h x n, row-major), b1 (h), W2 (n x h,
row-major), b2 (n)].  Loss over a batch of B pairs (x_b, t_b): the mean
squared error L = (1 / (B n)) sum_b ||y_b - t_b||^2.  Training uses Adam
(Kingma & Ba, 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def param_count(n: int, h: int) -> int:
    return h * n + h + n * h + n


def unpack(p: np.ndarray, n: int, h: int):
    p = np.asarray(p, np.float64)
    o = 0
    w1 = p[o:o + h * n].reshape(h, n); o += h * n
    b1 = p[o:o + h]; o += h
    w2 = p[o:o + n * h].reshape(n, h); o += n * h
    b2 = p[o:o + n]
    return w1, b1, w2, b2


def forward(p, x, n: int, h: int):
    """x: (B, n) -> (y (B, n), hidden activations (B, h))."""
    w1, b1, w2, b2 = unpack(p, n, h)
    a = np.tanh(np.asarray(x, np.float64) @ w1.T + b1)
    return a @ w2.T + b2, a


def loss_grad(p, x, t, n: int, h: int):
    """(loss, gradient with respect to the packed parameters)."""
    x = np.asarray(x, np.float64)
    t = np.asarray(t, np.float64)
    w1, b1, w2, b2 = unpack(p, n, h)
    y, a = forward(p, x, n, h)
    bsz = x.shape[0]
    r = y - t
    loss = float(np.sum(r * r) / (bsz * n))
    dy = 2.0 * r / (bsz * n)                 # dL/dy
    gw2 = dy.T @ a
    gb2 = dy.sum(axis=0)
    da = dy @ w2
    dz = da * (1.0 - a * a)                  # tanh'
    gw1 = dz.T @ x
    gb1 = dz.sum(axis=0)
    return loss, np.concatenate([gw1.ravel(), gb1, gw2.ravel(), gb2])


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step counts from 1); returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
