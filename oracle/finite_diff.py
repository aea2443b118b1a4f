"""Brute-force finite differences of <A> = Tr[A D(H)] (test infrastructure only).

Eq. (Suscept) defines chi^A_ij = d Tr[A D] / d H_ij.  For a symmetric H the
entries H_ij and H_ji move together, so a symmetric finite-difference direction
E = e_i e_j^T + e_j e_i^T (i != j) measures chi_ij + chi_ji = 2 chi_ij, and
E = e_i e_i^T measures chi_ii.  D(H) is taken from the eigendecomposition
(closed_form.density_matrix).
"""
from __future__ import annotations

import numpy as np

from .closed_form import density_matrix


def observable(h: np.ndarray, a: np.ndarray, nocc: int) -> float:
    d = density_matrix(h, nocc)
    return float(np.sum(np.asarray(a, np.float64) * d.T))


def directional(h, a, nocc, direction, step: float = 1e-5) -> float:
    """Central difference of Tr[A D(H + t E)] at t = 0."""
    h = np.asarray(h, np.float64)
    e = np.asarray(direction, np.float64)
    return (observable(h + step * e, a, nocc) - observable(h - step * e, a, nocc)) / (2 * step)


def susceptibility_fd(h, a, nocc, step: float = 1e-5) -> np.ndarray:
    """Every chi_ij by central differences (O(n^2) eigendecompositions; tiny n only)."""
    h = np.asarray(h, np.float64)
    n = h.shape[0]
    chi = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            e = np.zeros((n, n))
            e[i, j] = 1.0
            e[j, i] = 1.0
            g = directional(h, a, nocc, e, step)
            val = g if i == j else 0.5 * g
            chi[i, j] = chi[j, i] = val
    return chi
