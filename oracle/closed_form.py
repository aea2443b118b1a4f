"""Closed forms (FP64, CPU) — test infrastructure only.

Definitions followed
--------------------
* Sec. II: D = theta(mu I - H), the zero-temperature density matrix, with mu
  chosen so Tr D = N_occ.  For a gapped H this is the orthogonal projector onto
  the N_occ lowest eigenvectors.
* Eq. (Suscept): chi^A_ij = d Tr[A D] / d H_ij.  The paper's chi carries no
  spin factor; callers multiply by the spin factor s (s = 2 for a closed-shell
  system) themselves.
* Appendix, proof of the Equivalence relation: with H = V diag(lambda) V^T and
  the Loewner matrix L_ij = f[lambda_i, lambda_j] (divided differences of the
  occupation function f), Daleckii-Krein gives
      D^(1) = V (L o (V^T H1 V)) V^T,    chi^A = V (L o (V^T A V)) V^T.
  At zero temperature f is 1 on occupied and 0 on virtual states, so
  L_ij = (f_i - f_j) / (lambda_i - lambda_j) for f_i != f_j and 0 otherwise
  (the step function is flat away from mu, including the diagonal).
* Eq. (expectation) a0 = Tr[A D]; Eq. (direct) a1 = Tr[A D1];
  Eq. (dual) a1 = Tr[chi^A H1].
"""
from __future__ import annotations

import numpy as np


class GaplessError(ValueError):
    """Raised when the HOMO-LUMO gap at N_occ vanishes (D is not defined)."""


def _check(h: np.ndarray, nocc: int) -> np.ndarray:
    h = np.asarray(h, dtype=np.float64)
    if h.ndim != 2 or h.shape[0] != h.shape[1]:
        raise ValueError("H must be square")
    if not 0 <= nocc <= h.shape[0]:
        raise ValueError("need 0 <= nocc <= n")
    return h


def eigensystem(h: np.ndarray):
    """Ascending eigenvalues and orthonormal eigenvectors of symmetric h."""
    w, v = np.linalg.eigh(np.asarray(h, dtype=np.float64))
    return w, v


def occupations(n: int, nocc: int) -> np.ndarray:
    """Zero-temperature occupations f_i (1 for the nocc lowest states)."""
    f = np.zeros(n)
    f[:nocc] = 1.0
    return f


def gap(h: np.ndarray, nocc: int) -> float:
    h = _check(h, nocc)
    n = h.shape[0]
    if nocc in (0, n):
        return np.inf
    w = np.linalg.eigvalsh(h)
    return float(w[nocc] - w[nocc - 1])


def density_matrix(h: np.ndarray, nocc: int, tol: float = 1e-12) -> np.ndarray:
    """D = theta(mu I - H) (Sec. II): projector on the nocc lowest eigenvectors."""
    h = _check(h, nocc)
    n = h.shape[0]
    if nocc == 0:
        return np.zeros((n, n))
    if nocc == n:
        return np.eye(n)
    w, v = eigensystem(h)
    if w[nocc] - w[nocc - 1] <= tol * max(1.0, np.abs(w).max()):
        raise GaplessError("no gap at nocc: theta(mu I - H) is not defined")
    vo = v[:, :nocc]
    return vo @ vo.T


def loewner_step(w: np.ndarray, nocc: int) -> np.ndarray:
    """Divided differences of the zero-temperature occupation function."""
    f = occupations(w.size, nocc)
    df = f[:, None] - f[None, :]
    dl = w[:, None] - w[None, :]
    out = np.zeros_like(dl)
    mask = df != 0.0
    out[mask] = df[mask] / dl[mask]
    return out


def first_order_response(h: np.ndarray, pert: np.ndarray, nocc: int) -> np.ndarray:
    """Daleckii-Krein: d/dlambda theta(mu I - (H + lambda P)) = V (L o V^T P V) V^T.

    With P = H1 this is D^(1) (Eq. DM1's limit); with P = A it is the paper's
    chi^A (Eq. Suscept_Der / Equivalence).  No spin factor.
    """
    h = _check(h, nocc)
    n = h.shape[0]
    p = np.asarray(pert, dtype=np.float64)
    if nocc in (0, n):
        return np.zeros((n, n))
    w, v = eigensystem(h)
    if w[nocc] - w[nocc - 1] <= 1e-12 * max(1.0, np.abs(w).max()):
        raise GaplessError("no gap at nocc: the response is not defined")
    lmat = loewner_step(w, nocc)
    pt = v.T @ p @ v
    return v @ (lmat * pt) @ v.T


def first_order_responses(h: np.ndarray, perts: np.ndarray, nocc: int) -> np.ndarray:
    """first_order_response for a stack of perturbations (one eigendecomposition)."""
    h = _check(h, nocc)
    n = h.shape[0]
    perts = np.asarray(perts, dtype=np.float64)
    if nocc in (0, n):
        return np.zeros_like(perts)
    w, v = eigensystem(h)
    if w[nocc] - w[nocc - 1] <= 1e-12 * max(1.0, np.abs(w).max()):
        raise GaplessError("no gap at nocc: the response is not defined")
    lmat = loewner_step(w, nocc)
    return np.stack([v @ (lmat * (v.T @ p @ v)) @ v.T for p in perts])


def susceptibility(h: np.ndarray, a: np.ndarray, nocc: int, spin: float = 1.0) -> np.ndarray:
    """chi^A = s * dTr[A D]/dH (Eq. Suscept), via Daleckii-Krein."""
    return spin * first_order_response(h, a, nocc)


def density_response(h: np.ndarray, h1: np.ndarray, nocc: int) -> np.ndarray:
    """D^(1) for perturbation H1, via Daleckii-Krein (sum over states)."""
    return first_order_response(h, h1, nocc)


def expectation(a: np.ndarray, d: np.ndarray) -> float:
    """Eq. (expectation): a0 = Tr[A D]."""
    return float(np.sum(np.asarray(a, np.float64) * np.asarray(d, np.float64).T))


def response(chi: np.ndarray, h1s: np.ndarray) -> np.ndarray:
    """Eq. (dual): a1_p = Tr[chi H1_p] for a stack of perturbations."""
    chi = np.asarray(chi, np.float64)
    h1s = np.asarray(h1s, np.float64)
    if h1s.ndim == 2:
        h1s = h1s[None]
    return np.array([np.sum(chi * p.T) for p in h1s])


def rel_frobenius(x: np.ndarray, ref: np.ndarray) -> float:
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(np.asarray(x, np.float64) - ref)
    return float(num / den) if den > 0 else float(num)
