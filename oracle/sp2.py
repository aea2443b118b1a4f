"""SP2 recursion and its first-order / susceptibility sweeps in FP64 (CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every product is a full
FP64 matrix product; no symmetry tricks, no blocking, no fusion, so each
function can be read against the paper's equations.

Followed equations (arXiv 2409.17033)
-------------------------------------
* Eq. (DM0): X_1 = alpha I + beta H with alpha = emax/(emax-emin),
  beta = -1/(emax-emin); X_{n+1} = (1-sigma_n) X_n + sigma_n X_n^2; D = X_{M+1}.
* Eq. (DM1): Y_1 = beta H1; Y_{n+1} = (1-sigma_n) Y_n + sigma_n (Y_n X_n + X_n Y_n);
  D1 = Y_{M+1}.
* Eq. (DM2) (backward): Y_M = A; for n = M..1:
  Y_{n-1} = (1-sigma_n) Y_n + sigma_n (Y_n X_n + X_n Y_n); chi = beta Y_0.
* Eq. (DM3) (forward): Y_1 = beta A, the DM1 recursion; chi = Y_{M+1}.
* Eq. (DMSuscept) / Eq. (DMPert): DM3 / DM1 merged with DM0 so X_n is produced
  on the fly; a0 = Tr[D A].

Readings where the paper defers to a reference not reproduced in it
(the sigma choice and the stopping test, "Alg. 1" of the cited SP2 work):

* sigma_n: the paper's own statement (Sec. II) - pick the sign that puts
  Tr X_{n+1} closest to N_occ.  Tr X_n^2 = ||X_n||_F^2 for symmetric X_n, so
  both candidate traces, ||X||^2 and 2 Tr X - ||X||^2, are known from Tr X_n
  and ||X_n||_F^2 without forming a product.  Ties go to X^2 (sigma = +1).
* stop: with the idempotency error eps_n = ||X_n - X_n^2||_F^2 (= sum of
  (x - x^2)^2 over the eigenvalues, >= 0), stop at X_n once at least
  ``min_iter`` steps were taken and either eps_n <= idem_tol, or
  eps_n >= eps_{n-2} while eps_n < 1/64 (every state resolved to
  |x - x^2| < 1/8 and two further steps did not reduce the error: the
  arithmetic's rounding floor was reached).  The squared Frobenius measure
  cannot cancel between states above 1 and below 0 the way the trace
  measure Tr X - ||X||_F^2 does, so it stops at the floor instead of letting
  repeated same-sign steps amplify rounding noise.  ``min_iter`` (default 10)
  guards the first steps, where the error rises and falls while the spectrum
  is spread over [0, 1].
* unresolved: without a gap at N_occ some state stays near x = 1/2, eps_n
  never drops below 1/64 and the step limit reports not converged.
* bounds violation: a spectrum inside [0, 1] has 0 <= ||X||_F^2 <= n and
  0 <= Tr X <= n; an X_n outside these (or non-finite) means the supplied
  [emin, emax] did not enclose the spectrum of H and the recursion diverged.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


class NotConvergedError(RuntimeError):
    pass


class BoundsError(RuntimeError):
    pass


@dataclass
class SP2Trace:
    emin: float
    emax: float
    alpha: float
    beta: float
    sigmas: list = field(default_factory=list)   # sigma_n, n = 1..M
    traces: list = field(default_factory=list)   # Tr X_n, n = 1..M+1
    sqnorms: list = field(default_factory=list)  # ||X_n||_F^2
    errors: list = field(default_factory=list)   # eps_n = ||X_n - X_n^2||_F^2

    @property
    def m(self) -> int:
        return len(self.sigmas)


def gershgorin_bounds(h: np.ndarray) -> tuple[float, float]:
    """[emin, emax] enclosing the spectrum by Gershgorin's circle theorem."""
    h = np.asarray(h, np.float64)
    c = np.diag(h)
    r = np.abs(h).sum(axis=1) - np.abs(c)
    return float(np.min(c - r)), float(np.max(c + r))


def sp2_coefficients(emin: float, emax: float) -> tuple[float, float]:
    """alpha, beta of Eq. (DM0): spectrum of H mapped in reverse onto [0, 1]."""
    if not emax > emin:
        raise ValueError("need emax > emin")
    w = emax - emin
    return emax / w, -1.0 / w


def choose_sigma(tr: float, sq: float, nocc: float) -> int:
    """Sign whose update puts Tr X_{n+1} closest to N_occ (ties: X^2)."""
    t_square = sq                 # Tr X^2 = ||X||_F^2
    t_other = 2.0 * tr - sq       # Tr (2X - X^2)
    return 1 if abs(t_square - nocc) <= abs(t_other - nocc) else -1


def sp2_update(x: np.ndarray, sigma: int, x2: np.ndarray | None = None) -> np.ndarray:
    """X_{n+1} = (1 - sigma) X_n + sigma X_n^2  (Eq. DM0)."""
    return (1 - sigma) * x + sigma * (x @ x if x2 is None else x2)


def response_update(y: np.ndarray, x: np.ndarray, sigma: int) -> np.ndarray:
    """Y_{n+1} = (1 - sigma) Y_n + sigma (Y_n X_n + X_n Y_n)  (Eq. DM1/DM3)."""
    return (1 - sigma) * y + sigma * (y @ x + x @ y)


def _stats(x: np.ndarray) -> tuple[float, float]:
    return float(np.trace(x)), float(np.sum(x * x))


UNRESOLVED = 1.0 / 64.0   # eps above this: some state still has |x - x^2| >= 1/8


def should_stop(errors: list, steps: int, min_iter: int, idem_tol: float) -> bool:
    """Stopping test for the newest iterate (errors[-1] = eps_n, steps = n - 1)."""
    if steps < min_iter:
        return False
    e = errors[-1]
    if e <= idem_tol:
        return True
    return len(errors) >= 3 and e >= errors[-3] and e < UNRESOLVED


def _check_bounds(tr: float, sq: float, n: int) -> None:
    if not (np.isfinite(tr) and np.isfinite(sq)):
        raise BoundsError("non-finite iterate: spectrum bounds do not enclose H")
    if sq > n + 1.0 or tr < -1.0 or tr > n + 1.0:
        raise BoundsError("iterate left [0,1]: spectrum bounds do not enclose H")


def _trivial(n: int, nocc: int):
    if nocc == 0:
        return np.zeros((n, n))
    if nocc == n:
        return np.eye(n)
    return None


def sp2_merged(h: np.ndarray, ys: list, nocc: int, emin: float | None = None,
               emax: float | None = None, max_iter: int = 200, min_iter: int = 10,
               idem_tol: float = 0.0):
    """Eq. (DM0) merged with the response recursion for each Y_1 in ``ys``.

    ``ys`` holds the *unscaled* first-order matrices (A for Eq. DMSuscept,
    H1 for Eq. DMPert); Y_1 = beta * ys[k].  Returns (D, [Y_{M+1}], trace).
    """
    h = np.asarray(h, np.float64)
    n = h.shape[0]
    if emin is None or emax is None:
        emin, emax = gershgorin_bounds(h)
    alpha, beta = sp2_coefficients(emin, emax)
    tr = SP2Trace(emin, emax, alpha, beta)
    triv = _trivial(n, nocc)
    if triv is not None:
        return triv, [np.zeros((n, n)) for _ in ys], tr
    x = alpha * np.eye(n) + beta * h
    yv = [beta * np.asarray(y, np.float64) for y in ys]
    for step in range(max_iter + 1):
        t, q = _stats(x)
        _check_bounds(t, q, n)
        x2 = x @ x
        tr.traces.append(t)
        tr.sqnorms.append(q)
        tr.errors.append(float(np.sum((x - x2) ** 2)))
        if should_stop(tr.errors, step, min_iter, idem_tol):
            return x, yv, tr
        if step == max_iter:
            break
        s = choose_sigma(t, q, nocc)
        tr.sigmas.append(s)
        yv = [response_update(y, x, s) for y in yv]
        x = sp2_update(x, s, x2)
    raise NotConvergedError(f"SP2 did not converge in {max_iter} steps")


def sp2_density(h, nocc, emin=None, emax=None, **kw):
    """Eq. (DM0): D = X_{M+1}.  Returns (D, trace)."""
    d, _, tr = sp2_merged(h, [], nocc, emin, emax, **kw)
    return d, tr


def sp2_susceptibility(h, a, nocc, emin=None, emax=None, spin: float = 1.0, **kw):
    """Eq. (DMSuscept): returns (D, s * chi^A, a0 = s Tr[D A], trace)."""
    d, (y,), tr = sp2_merged(h, [a], nocc, emin, emax, **kw)
    a0 = spin * float(np.sum(d * np.asarray(a, np.float64).T))
    return d, spin * y, a0, tr


def sp2_density_response(h, h1, nocc, emin=None, emax=None, **kw):
    """Eq. (DMPert): returns (D, D^(1), trace)."""
    d, (y,), tr = sp2_merged(h, [h1], nocc, emin, emax, **kw)
    return d, y, tr


def sp2_sequence(h: np.ndarray, sigmas, emin: float, emax: float):
    """X_1..X_{M+1} of Eq. (DM0) for a *given* sigma sequence (no stop test)."""
    h = np.asarray(h, np.float64)
    n = h.shape[0]
    alpha, beta = sp2_coefficients(emin, emax)
    xs = [alpha * np.eye(n) + beta * h]
    for s in sigmas:
        xs.append(sp2_update(xs[-1], s))
    return xs, beta


def forward_sweep(xs, sigmas, beta: float, y0: np.ndarray) -> np.ndarray:
    """Eq. (DM3) / Eq. (DM1) over a stored X sequence: Y_1 = beta y0 -> Y_{M+1}."""
    y = beta * np.asarray(y0, np.float64)
    for n, s in enumerate(sigmas):
        y = response_update(y, xs[n], s)
    return y


def backward_sweep(xs, sigmas, beta: float, a: np.ndarray) -> np.ndarray:
    """Eq. (DM2): Y_M = A, Y_{n-1} from Y_n with X_n, sigma_n for n = M..1; chi = beta Y_0."""
    y = np.asarray(a, np.float64)
    for n in range(len(sigmas) - 1, -1, -1):
        y = response_update(y, xs[n], sigmas[n])
    return beta * y


def sp2_backward_susceptibility(h, a, nocc, emin=None, emax=None, spin=1.0, **kw):
    """Susceptibility by the backward expansion, Eq. (DM2), after running
    Eq. (DM0) to find M and the sigma sequence and storing every X_n."""
    h = np.asarray(h, np.float64)
    n = h.shape[0]
    d, tr = sp2_density(h, nocc, emin, emax, **kw)
    if nocc in (0, n):
        return d, np.zeros((n, n)), tr
    xs, beta = sp2_sequence(h, tr.sigmas, tr.emin, tr.emax)
    return d, spin * backward_sweep(xs, tr.sigmas, beta, a), tr
