"""FP64 oracle for the self-consistent susceptibility (Eq. CP_SCF) and the
self-consistent density-matrix response (Eq. DM_CP_SCF), Sec. V.C and the
Appendix, at zero temperature in an orthonormal basis (Z = I, mu_1 = 0).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Model.  The self-consistent field is an on-site interaction,
    H = H0 + diag(U_i (n_i - n0_i)),   n = s diag(D),   n0 = s diag(D(H0)),
so H0 is the converged ground state and only the response is
self-consistent.  The linearised field of a density-matrix change X is
    G(X) = diag(U_i s X_ii),
which is self-adjoint (Tr[X G(Y)] = Tr[Y G(X)]), the property the dual
(susceptibility) formulation needs.

With L the non-interacting first-order response (Daleckii-Krein, spin-less):
    Eq. CP_SCF     chi' = L[A + G(chi')],       chi = s chi'
    Eq. DM_CP_SCF  D1   = L[H1 + G(D1)],        a1  = s Tr[A D1] = Tr[chi H1]
Both are iterated exactly as the paper writes them (linear mixing with a
constant c_mix); G only reads the diagonal, so the iteration state is the
N-vector v = diag(chi') (or diag(D1)).
"""
from __future__ import annotations

import numpy as np

from .closed_form import GaplessError, eigensystem, loewner_step


class FirstOrder:
    """The linear map B -> L[B] = V (Lw o V^T B V) V^T for a fixed H0
    (Daleckii-Krein), with the eigendecomposition done once."""

    def __init__(self, h0: np.ndarray, nocc: int):
        h0 = np.asarray(h0, np.float64)
        self.n = h0.shape[0]
        self.nocc = nocc
        w, v = eigensystem(h0)
        if 0 < nocc < self.n and w[nocc] - w[nocc - 1] <= 1e-12 * max(1.0, np.abs(w).max()):
            raise GaplessError("no gap at nocc")
        self.w, self.v = w, v
        self.lw = loewner_step(w, nocc)

    def __call__(self, b: np.ndarray) -> np.ndarray:
        if self.nocc in (0, self.n):
            return np.zeros((self.n, self.n))
        bt = self.v.T @ np.asarray(b, np.float64) @ self.v
        return self.v @ (self.lw * bt) @ self.v.T

    def density(self) -> np.ndarray:
        vo = self.v[:, :self.nocc]
        return vo @ vo.T


def onsite_field(x: np.ndarray, u: np.ndarray, spin: float) -> np.ndarray:
    """G(X) = diag(U_i s X_ii)."""
    return np.diag(np.asarray(u, np.float64) * spin * np.diag(np.asarray(x, np.float64)))


def _scf_linear(lmap: FirstOrder, source: np.ndarray, u: np.ndarray, spin: float, mix: float,
                tol: float, max_iter: int):
    """X = L[source + G(X)] by the paper's loop: X_new = L[source + G(X_old)],
    dX = X_new - X_old, X = X_old + c_mix dX, until ||dX||_F <= tol."""
    x = np.zeros((lmap.n, lmap.n))
    history = []
    for it in range(1, max_iter + 1):
        x_new = lmap(source + onsite_field(x, u, spin))
        dx = x_new - x
        history.append(float(np.linalg.norm(dx)))
        x = x + mix * dx
        if history[-1] <= tol:
            return x, it, history
    raise RuntimeError(f"SCF response did not converge in {max_iter} iterations")


def scf_susceptibility(h0, a, u, nocc, spin: float = 2.0, mix: float = 0.3, tol: float = 1e-13,
                       max_iter: int = 5000):
    """Eq. CP_SCF: returns (chi = s chi', iterations, ||d chi'|| history)."""
    lmap = FirstOrder(h0, nocc)
    x, it, hist = _scf_linear(lmap, np.asarray(a, np.float64), u, spin, mix, tol, max_iter)
    return spin * x, it, hist


def scf_density_response(h0, h1, u, nocc, spin: float = 2.0, mix: float = 0.3, tol: float = 1e-13,
                         max_iter: int = 5000):
    """Eq. DM_CP_SCF: returns (D1 (spin-less), iterations, history)."""
    lmap = FirstOrder(h0, nocc)
    return _scf_linear(lmap, np.asarray(h1, np.float64), u, spin, mix, tol, max_iter)


def scf_fixed_point_map(h0, a, u, nocc, spin: float = 2.0):
    """F(v) = diag(L[A + diag(U s v)]) on the diagonal state v = diag(chi'),
    and the exact fixed point v* (its Jacobian J = d F/d v is formed column
    by column: F is affine).  For small n only."""
    lmap = FirstOrder(h0, nocc)
    n = lmap.n
    f0 = np.diag(lmap(np.asarray(a, np.float64))).copy()
    jac = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        jac[:, j] = np.diag(lmap(np.diag(np.asarray(u, np.float64) * spin * e)))
    vstar = np.linalg.solve(np.eye(n) - jac, f0)
    return f0, jac, vstar


def scf_ground_state(h0, u, nocc, spin: float = 2.0, h_ext=None, mix: float = 0.5, tol: float = 1e-15,
                     max_iter: int = 20000):
    """Self-consistent ground state of H = H0 + h_ext + diag(U (n - n0)),
    n = s diag D(H), n0 = s diag D(H0); returns D.  With h_ext = 0 the answer
    is D(H0).  Plain mixing on n; for small systems and finite differences."""
    from .closed_form import density_matrix
    h0 = np.asarray(h0, np.float64)
    u = np.asarray(u, np.float64)
    n0 = spin * np.diag(density_matrix(h0, nocc))
    hx = h0 + (0.0 if h_ext is None else np.asarray(h_ext, np.float64))
    n_cur = n0.copy()
    for _ in range(max_iter):
        d = density_matrix(hx + np.diag(u * (n_cur - n0)), nocc)
        n_new = spin * np.diag(d)
        if np.max(np.abs(n_new - n_cur)) <= tol:
            return density_matrix(hx + np.diag(u * (n_new - n0)), nocc)
        n_cur = n_cur + mix * (n_new - n_cur)
    raise RuntimeError("SCF ground state did not converge")
