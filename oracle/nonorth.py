"""FP64 oracle for a non-orthonormal basis (Sec. V.A) — TEST INFRASTRUCTURE ONLY
(see oracle/__init__.py).

With an overlap matrix S and an inverse factor Z (Z^T S Z = I; Z = S^{-1/2}
for Loewdin orthonormalisation, Z = L^{-T} for the Cholesky factor S = L L^T)
the orthonormal representations are congruences:
    H_perp = Z^T H Z,   A_perp = Z^T A Z,   D = Z D_perp Z^T,
    D_perp = theta(mu I - H_perp)  (Tr D_perp = N_occ),
and a0 = Tr[A D] = Tr[A_perp D_perp] by cyclic invariance.  The
susceptibility of the orthonormal problem is chi_perp = s dTr[A_perp D_perp]/dH_perp
(Eq. Suscept in the orthonormal basis); for a perturbation of H at fixed S,
dH_perp = Z^T dH Z, so the atomic-orbital susceptibility that contracts with
dH is chi_ao = Z chi_perp Z^T (Tr[chi_perp Z^T dH Z] = Tr[Z chi_perp Z^T dH]).
"""
from __future__ import annotations

import numpy as np

from . import closed_form as cf


def loewdin_factor(s: np.ndarray) -> np.ndarray:
    """Z = S^{-1/2} (symmetric) from the eigendecomposition of S."""
    w, v = np.linalg.eigh(np.asarray(s, np.float64))
    if w[0] <= 0:
        raise ValueError("S is not positive definite")
    return (v / np.sqrt(w)) @ v.T


def cholesky_factor(s: np.ndarray) -> np.ndarray:
    """Z = L^{-T} for S = L L^T (upper triangular Z)."""
    ell = np.linalg.cholesky(np.asarray(s, np.float64))
    return np.linalg.inv(ell).T


def congruence(z: np.ndarray, m: np.ndarray) -> np.ndarray:
    """Z^T M Z."""
    z = np.asarray(z, np.float64)
    return z.T @ np.asarray(m, np.float64) @ z


def nonorth_response(h, z, a, nocc: int, spin: float = 2.0):
    """(D, chi_perp, chi_ao, a0) for one observable A in the basis with inverse
    factor Z: D = Z D_perp Z^T, chi_perp = s * DK(H_perp, A_perp),
    chi_ao = Z chi_perp Z^T, a0 = s Tr[A D]."""
    z = np.asarray(z, np.float64)
    hp = congruence(z, h)
    ap = congruence(z, a)
    dp = cf.density_matrix(hp, nocc)
    chi_p = spin * cf.first_order_response(hp, ap, nocc)
    d = z @ dp @ z.T
    return d, chi_p, z @ chi_p @ z.T, spin * float(np.sum(np.asarray(a, np.float64) * d))


def generalized_density(h, s, nocc: int) -> np.ndarray:
    """D = C_occ C_occ^T from the generalised eigenproblem H C = S C e with
    C^T S C = I (no inverse factor involved)."""
    import scipy.linalg
    _, c = scipy.linalg.eigh(np.asarray(h, np.float64), np.asarray(s, np.float64))
    co = c[:, :nocc]
    return co @ co.T
