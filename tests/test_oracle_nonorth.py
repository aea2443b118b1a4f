"""Pins of the non-orthonormal-basis oracle (Sec. V.A), independent of its
own formulas: the identity factor reduces to the orthonormal closed form;
the density from the generalised eigenproblem H C = S C e (no inverse
factor) equals Z D_perp Z^T for both the Loewdin and the Cholesky factor;
a0 = Tr[A D] = Tr[A_perp D_perp]; chi_ao does not depend on the choice of Z
and equals brute-force central differences of s Tr[A D(H)] at fixed S."""
import numpy as np

from oracle import closed_form as cf
from oracle import nonorth as no


def _case(n=8, nocc=3, seed=0):
    rng = np.random.default_rng(seed)
    h = rng.normal(size=(n, n))
    h = 0.5 * (h + h.T)
    w, v = np.linalg.eigh(h)
    w[nocc:] += 1.0                                   # open a gap at nocc
    h = (v * w) @ v.T
    g = rng.normal(size=(n, n)) * 0.2
    s = np.eye(n) + 0.5 * (g + g.T) @ (g + g.T).T / n  # SPD overlap near I
    a = rng.normal(size=(n, n))
    return h, s, 0.5 * (a + a.T), nocc


def test_identity_factor_is_orthonormal_case():
    h, _, a, nocc = _case()
    d, chi_p, chi_ao, a0 = no.nonorth_response(h, np.eye(h.shape[0]), a, nocc, spin=2.0)
    np.testing.assert_allclose(d, cf.density_matrix(h, nocc), atol=1e-12)
    np.testing.assert_allclose(chi_p, cf.susceptibility(h, a, nocc, spin=2.0), atol=1e-12)
    np.testing.assert_allclose(chi_ao, chi_p, atol=1e-12)


def test_inverse_factors_satisfy_definition():
    _, s, _, _ = _case()
    for z in (no.loewdin_factor(s), no.cholesky_factor(s)):
        np.testing.assert_allclose(z.T @ s @ z, np.eye(s.shape[0]), atol=1e-12)
    np.testing.assert_allclose(no.loewdin_factor(s), no.loewdin_factor(s).T, atol=1e-13)


def test_density_matches_generalised_eigenproblem():
    h, s, a, nocc = _case()
    dg = no.generalized_density(h, s, nocc)
    for z in (no.loewdin_factor(s), no.cholesky_factor(s)):
        d, _, _, a0 = no.nonorth_response(h, z, a, nocc, spin=2.0)
        np.testing.assert_allclose(d, dg, atol=1e-11)
        # a0 = s Tr[A D] = s Tr[A_perp D_perp]
        dp = cf.density_matrix(no.congruence(z, h), nocc)
        assert abs(a0 - 2.0 * np.sum(no.congruence(z, a) * dp)) < 1e-11
    # D S D = D (idempotent in the S metric), Tr[S D] = N_occ
    np.testing.assert_allclose(dg @ s @ dg, dg, atol=1e-11)
    assert abs(np.trace(s @ dg) - nocc) < 1e-11


def test_chi_ao_is_the_derivative_at_fixed_overlap():
    h, s, a, nocc = _case(n=6, nocc=2, seed=3)
    _, _, chi_l, _ = no.nonorth_response(h, no.loewdin_factor(s), a, nocc, spin=2.0)
    _, _, chi_c, _ = no.nonorth_response(h, no.cholesky_factor(s), a, nocc, spin=2.0)
    np.testing.assert_allclose(chi_l, chi_c, atol=1e-10)
    n, step = h.shape[0], 1e-5
    fd = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            e = np.zeros((n, n))
            e[i, j] = e[j, i] = 1.0
            fp = 2.0 * np.sum(a * no.generalized_density(h + step * e, s, nocc))
            fm = 2.0 * np.sum(a * no.generalized_density(h - step * e, s, nocc))
            g = (fp - fm) / (2 * step)
            fd[i, j] = fd[j, i] = g if i == j else g / 2.0   # symmetric direction moves two entries
    np.testing.assert_allclose(chi_l, fd, atol=1e-7)
