"""FP64 oracle for fractional occupation at finite electronic temperature
(Sec. V.B) — TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Definitions
-----------
* Fermi function of H: D = f(H) = (exp(beta (H - mu I)) + I)^{-1},
  beta = 1 / (k_B T_e).  Canonical ensemble: mu such that Tr D = N_occ.
* Temperature-dependent susceptibility (Sec. V.B): the derivative of
  f(H + lambda (A + mu_1 I)) at lambda = 0, with mu_1 the first-order shift of
  the chemical potential that keeps the electron count (Tr chi = 0).
  Daleckii-Krein with f'(w) = -beta f (1 - f): chi' = V (L o (V^T (A + mu_1 I) V)) V^T,
  L_ij = (f_i - f_j) / (w_i - w_j), L_ii = f'(w_i), and
  mu_1 = - sum_i L_ii A~_ii / sum_i L_ii  (A~ = V^T A V).
* Recursive Fermi-operator expansion (Niklasson, Phys. Rev. B 66, 155115
  (2002)): with t = 1 / (1 + e^z), t^2 / (t^2 + (1 - t)^2) = 1 / (1 + e^{2z}),
  so m doubling steps X_{k+1} = X_k^2 [X_k^2 + (I - X_k)^2]^{-1} take
  X_0 = f at temperature 2^m T_e to f at T_e; at the high temperature the
  Fermi function is linear to third order: X_0 = I/2 - (beta / 2^{m+2})(H - mu I).
  Its first-order response Y_k = dX_k/dlambda follows by the product rule,
  Y_{k+1} = (dP - X_{k+1} dQ) Q^{-1} with P = X_k^2, Q = P + (I - X_k)^2,
  dP = Y_k X_k + X_k Y_k, dQ = 2 dP - 2 Y_k, Y_0 = -(beta / 2^{m+2}) B.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expit

from .closed_form import eigensystem


def occupations(w: np.ndarray, mu: float, beta: float) -> np.ndarray:
    """f_i = 1 / (1 + exp(beta (w_i - mu))), evaluated without overflow."""
    return expit(-beta * (np.asarray(w, np.float64) - mu))


def chemical_potential(w: np.ndarray, nocc: float, beta: float, tol: float = 1e-14) -> float:
    """mu with sum_i f_i = nocc, by bisection (the count is monotone in mu)."""
    w = np.asarray(w, np.float64)
    lo, hi = w[0] - 50.0 / beta - 1.0, w[-1] + 50.0 / beta + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if occupations(w, mid, beta).sum() < nocc:
            lo = mid
        else:
            hi = mid
        if hi - lo <= tol * max(1.0, abs(mid)):
            break
    return 0.5 * (lo + hi)


def fermi_density(h, nocc: float, beta: float):
    """(D, mu) for the canonical ensemble."""
    w, v = eigensystem(h)
    mu = chemical_potential(w, nocc, beta)
    return (v * occupations(w, mu, beta)) @ v.T, mu


def loewner_fermi(w: np.ndarray, mu: float, beta: float) -> np.ndarray:
    """Divided differences of f; the derivative -beta f (1 - f) on (near-)equal pairs."""
    w = np.asarray(w, np.float64)
    f = occupations(w, mu, beta)
    dw = w[:, None] - w[None, :]
    df = f[:, None] - f[None, :]
    fbar = occupations(0.5 * (w[:, None] + w[None, :]), mu, beta)
    close = np.abs(dw) < 1e-9 / max(beta, 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        lw = np.where(close, -beta * fbar * (1.0 - fbar), df / np.where(close, 1.0, dw))
    return lw


def fermi_susceptibility(h, a, nocc: float, beta: float, spin: float = 1.0, canonical: bool = True):
    """(chi = s chi', mu, mu_1) for one observable A."""
    w, v = eigensystem(h)
    mu = chemical_potential(w, nocc, beta)
    lw = loewner_fermi(w, mu, beta)
    at = v.T @ np.asarray(a, np.float64) @ v
    mu1 = 0.0
    if canonical:
        d = np.diag(lw)
        mu1 = -float(d @ np.diag(at)) / float(d.sum())
    chi = v @ (lw * (at + mu1 * np.eye(len(w)))) @ v.T
    return spin * chi, mu, mu1


def recursive_fermi(h, mu: float, beta: float, m: int, b=None):
    """The expansion run for m doubling steps at a given mu; with b (a
    perturbation direction) also its first-order response.  Returns (X_m, Y_m)."""
    h = np.asarray(h, np.float64)
    n = h.shape[0]
    eye = np.eye(n)
    c = beta / 2.0 ** (m + 2)
    x = 0.5 * eye - c * (h - mu * eye)
    y = None if b is None else -c * np.asarray(b, np.float64)
    for _ in range(m):
        p = x @ x
        q = p + (eye - x) @ (eye - x)
        x_new = np.linalg.solve(q, p)          # P Q^{-1} = Q^{-1} P (both functions of X)
        if y is not None:
            dp = y @ x + x @ y
            dq = 2.0 * dp - 2.0 * y
            y = np.linalg.solve(q.T, (dp - x_new @ dq).T).T   # (dP - X_{k+1} dQ) Q^{-1}
        x = x_new
    return x, y
