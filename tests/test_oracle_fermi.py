"""Pins of the finite-temperature oracle (Sec. V.B) that do not reuse its
formulas: the Fermi function of a 2 x 2 system by hand; the electron count
and its low-temperature limit (the zero-temperature projector); brute-force
central differences of Tr[A f(H + lambda A)] with the chemical potential
re-solved at every lambda (the canonical susceptibility is that derivative);
the doubling recursion against the closed form and its response against
finite differences of the recursion itself."""
import numpy as np

from oracle import closed_form as cf
from oracle import fermi as fo


def _case(n=10, nocc=4, seed=0):
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(n, n))
    h = 0.5 * (g + g.T) / np.sqrt(n)
    a = rng.normal(size=(n, n))
    return h, 0.5 * (a + a.T), nocc


def test_two_level_by_hand():
    """H = diag(-0.1, 0.3), one electron, beta = 10: f_i = 1/(1+e^{beta(e_i - mu)})
    with f_1 + f_2 = 1, i.e. mu = 0.1 and f = (1/(1+e^{-2}), 1/(1+e^{2}))."""
    d, mu = fo.fermi_density(np.diag([-0.1, 0.3]), 1.0, 10.0)
    assert abs(mu - 0.1) < 1e-12
    np.testing.assert_allclose(np.diag(d), [1 / (1 + np.exp(-2.0)), 1 / (1 + np.exp(2.0))], rtol=1e-13)


def test_count_and_zero_temperature_limit():
    h, _, nocc = _case()
    d, _ = fo.fermi_density(h, nocc, 30.0)
    assert abs(np.trace(d) - nocc) < 1e-12
    w = np.linalg.eigvalsh(h)
    if w[nocc] - w[nocc - 1] > 0.05:
        d_cold, _ = fo.fermi_density(h, nocc, 5000.0)
        np.testing.assert_allclose(d_cold, cf.density_matrix(h, nocc), atol=1e-12)


def test_canonical_susceptibility_is_the_derivative():
    h, a, nocc = _case(n=8, nocc=3, seed=2)
    beta, lam = 20.0, 1e-5
    chi, _, _ = fo.fermi_susceptibility(h, a, nocc, beta)
    # chi = d/dlambda f(H + lambda A) with mu(lambda) re-solved: Tr[B chi] for a direction B
    rng = np.random.default_rng(5)
    for _ in range(3):
        b = rng.normal(size=h.shape)
        b = 0.5 * (b + b.T)
        dp, _ = fo.fermi_density(h + lam * a, nocc, beta)
        dm, _ = fo.fermi_density(h - lam * a, nocc, beta)
        fd = np.sum(b * (dp - dm)) / (2 * lam)
        assert abs(np.sum(b * chi) - fd) < 1e-7 * max(1.0, abs(fd))
    assert abs(np.trace(chi)) < 1e-12          # the electron count does not move
    np.testing.assert_allclose(chi, chi.T, atol=1e-13)


def test_grand_canonical_duality():
    """Without the mu shift, f'(H)[.] is self-adjoint: Tr[A f'[B]] = Tr[f'[A] B]."""
    h, a, nocc = _case(n=9, nocc=4, seed=3)
    rng = np.random.default_rng(1)
    b = rng.normal(size=h.shape)
    b = 0.5 * (b + b.T)
    ca, _, _ = fo.fermi_susceptibility(h, a, nocc, 15.0, canonical=False)
    cb, _, _ = fo.fermi_susceptibility(h, b, nocc, 15.0, canonical=False)
    assert abs(np.sum(a * cb) - np.sum(ca * b)) < 1e-12


def test_recursion_reaches_fermi_dirac():
    h, a, nocc = _case(n=12, nocc=5, seed=4)
    beta = 40.0
    d, mu = fo.fermi_density(h, nocc, beta)
    for m, tol in ((10, 1e-5), (16, 1e-10)):
        x, _ = fo.recursive_fermi(h, mu, beta, m)
        assert np.abs(x - d).max() < tol, m
    # response of the recursion = its own central difference (step 1e-5:
    # truncation ~step^2 and the rounding of X amplified by the 2^16 doubling
    # both stay near 5e-8 of max|Y| ~ 2)
    x, y = fo.recursive_fermi(h, mu, beta, 16, b=a)
    step = 1e-5
    xp, _ = fo.recursive_fermi(h + step * a, mu, beta, 16)
    xm, _ = fo.recursive_fermi(h - step * a, mu, beta, 16)
    np.testing.assert_allclose(y, (xp - xm) / (2 * step), atol=2e-7)
    # and the grand-canonical susceptibility up to the linearised start: its
    # slope -1/4 differs from the exact -e^eps / (1 + e^eps)^2 by ~eps^2 / 16,
    # eps = beta max|w - mu| / 2^m (relative ~3e-7 at m = 16, ~1e-9 at m = 20)
    gc, _, _ = fo.fermi_susceptibility(h, a, nocc, beta, canonical=False)
    w = np.linalg.eigvalsh(h)
    for m in (16, 20):
        _, y = fo.recursive_fermi(h, mu, beta, m, b=a)
        eps = beta * np.abs(w - mu).max() / 2.0 ** m
        assert np.abs(y - gc).max() <= 4 * eps ** 2 * np.abs(gc).max(), m
