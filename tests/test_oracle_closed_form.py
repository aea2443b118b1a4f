"""Pins for the closed-form oracle (CPU only).

Each test checks the oracle against something other than itself: a hand
derivation, textbook perturbation theory, brute-force finite differences, a
matrix built from a known spectrum, or an identity the definitions force.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf
from oracle import finite_diff as fd

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_two_level_golden():
    g = _load("two_level.json")
    h, a = np.array(g["H"]), np.array(g["A"])
    d = cf.density_matrix(h, g["nocc"])
    chi = cf.susceptibility(h, a, g["nocc"])
    np.testing.assert_allclose(d, g["D"], atol=1e-14)
    np.testing.assert_allclose(chi, g["chi"], atol=1e-14)
    assert abs(cf.expectation(a, d) - g["a0"]) < 1e-14
    assert abs(cf.response(chi, a)[0] - g["response_to_A"]) < 1e-14


def test_diagonal_rspt_golden():
    g = _load("diagonal_rspt.json")
    h = np.diag(g["H_diag"])
    chi = cf.susceptibility(h, np.array(g["A"]), g["nocc"])
    np.testing.assert_allclose(chi, g["chi"], atol=1e-14)


def _two_by_two_closed_form(a, c, d, amat):
    """Hand derivation for N=2, N_occ=1 without any eigendecomposition.

    K = H - (a+d)/2 I is traceless with K^2 = R^2 I, R = sqrt(((a-d)/2)^2 + c^2).
    The lower-state projector is D = (I - K/R)/2.  Differentiating
    Tr[A D] = Tr[A]/2 - Tr[A K]/(2R) along a symmetric E, with dR = Tr[K E]/(2R),
    gives chi = -Abar/(2R) + Tr[A K] K/(4 R^3), Abar = A - Tr[A]/2 I.
    """
    k = np.array([[(a - d) / 2, c], [c, (d - a) / 2]])
    r = np.hypot((a - d) / 2, c)
    dmat = 0.5 * (np.eye(2) - k / r)
    abar = amat - 0.5 * np.trace(amat) * np.eye(2)
    chi = -abar / (2 * r) + np.trace(amat @ k) * k / (4 * r ** 3)
    return dmat, chi


@pytest.mark.parametrize("seed", range(6))
def test_two_by_two_analytic(seed):
    rng = np.random.default_rng(seed)
    a, c, d = rng.normal(size=3)
    amat = rng.normal(size=(2, 2))
    amat = amat + amat.T
    h = np.array([[a, c], [c, d]])
    dref, chiref = _two_by_two_closed_form(a, c, d, amat)
    np.testing.assert_allclose(cf.density_matrix(h, 1), dref, atol=1e-13)
    np.testing.assert_allclose(cf.susceptibility(h, amat, 1), chiref, atol=1e-12)


@pytest.mark.parametrize("n,nocc", [(5, 2), (8, 3), (9, 5)])
def test_diagonal_h_is_textbook_first_order(n, nocc):
    rng = np.random.default_rng(n)
    e = rng.permutation(np.linspace(-2, 2, n))       # unsorted site energies
    a = rng.normal(size=(n, n))
    a = a + a.T
    chi = cf.susceptibility(np.diag(e), a, nocc)
    occ = np.argsort(e)[:nocc]
    vir = np.argsort(e)[nocc:]
    ref = np.zeros((n, n))
    for i in occ:
        for v in vir:
            ref[i, v] = ref[v, i] = a[i, v] / (e[i] - e[v])
    np.testing.assert_allclose(chi, ref, atol=1e-13)


@pytest.mark.parametrize("n,nocc", [(4, 2), (6, 2), (7, 4)])
def test_susceptibility_against_brute_force_fd(n, nocc):
    h, _, _ = W.known_spectrum(n, nocc, gap=0.5, seed=n)
    rng = np.random.default_rng(100 + n)
    a = rng.normal(size=(n, n))
    a = a + a.T
    chi = cf.susceptibility(h, a, nocc)
    chi_fd = fd.susceptibility_fd(h, a, nocc, step=1e-5)
    assert np.max(np.abs(chi - chi_fd)) < 1e-7 * max(1.0, np.max(np.abs(chi)))


@pytest.mark.parametrize("n,nocc", [(16, 5), (40, 20), (64, 63), (64, 1)])
def test_density_matrix_from_known_spectrum(n, nocc):
    h, w, q = W.known_spectrum(n, nocc, seed=3)
    d = cf.density_matrix(h, nocc)
    np.testing.assert_allclose(d, q[:, :nocc] @ q[:, :nocc].T, atol=1e-12)
    # lowest-energy projector: Tr[H D] is the sum of the nocc smallest eigenvalues
    assert abs(np.trace(h @ d) - np.sum(w[:nocc])) < 1e-11


def test_density_matrix_identities_config1():
    wl = W.dense_gapped(128)
    h = wl.H.astype(np.float64)
    d = cf.density_matrix(h, wl.nocc)
    assert np.linalg.norm(d @ d - d) < 1e-12 * np.sqrt(wl.nocc)
    assert abs(np.trace(d) - wl.nocc) < 1e-11
    assert np.linalg.norm(h @ d - d @ h) < 1e-12 * np.linalg.norm(h)


def test_susceptibility_identities_config1():
    wl = W.dense_gapped(128)
    h = wl.H.astype(np.float64)
    a = wl.A[0].astype(np.float64)
    d = cf.density_matrix(h, wl.nocc)
    chi = cf.susceptibility(h, a, wl.nocc)
    nrm = np.linalg.norm(chi)
    # symmetric, traceless (shift invariance: H -> H + c I leaves D unchanged)
    assert np.linalg.norm(chi - chi.T) < 1e-13 * nrm
    assert abs(np.trace(chi)) < 1e-12 * nrm * np.sqrt(wl.n)
    # [H, chi] = [D, A]: from (lambda_i - lambda_j) L_ij = f_i - f_j
    lhs = h @ chi - chi @ h
    rhs = d @ a - a @ d
    assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(rhs)
    # only occupied-virtual blocks: chi = D chi (I-D) + (I-D) chi D
    i = np.eye(wl.n)
    ov = d @ chi @ (i - d) + (i - d) @ chi @ d
    assert np.linalg.norm(chi - ov) < 1e-12 * nrm


def test_hadamard_trace_symmetry():
    """Tr[(L o X) Y] = Tr[(L o Y) X] for symmetric L, X, Y (Appendix, Equivalence proof)."""
    wl = W.dense_gapped(128)
    w = np.linalg.eigvalsh(wl.H.astype(np.float64))
    lmat = cf.loewner_step(w, wl.nocc)
    assert np.allclose(lmat, lmat.T)
    rng = np.random.default_rng(5)
    x = rng.normal(size=(128, 128)); x += x.T
    y = rng.normal(size=(128, 128)); y += y.T
    assert abs(np.trace((lmat * x) @ y) - np.trace((lmat * y) @ x)) < 1e-10


def test_duality_closed_form_config1():
    """Eq. (Equivalence): Tr[A D1] = Tr[chi^A H1] for each of the 8 perturbations."""
    wl = W.dense_gapped(128)
    h = wl.H.astype(np.float64)
    a = wl.A[0].astype(np.float64)
    chi = cf.susceptibility(h, a, wl.nocc, spin=2.0)
    r_dual = cf.response(chi, wl.H1)
    r_direct = np.array([2.0 * cf.expectation(a, cf.density_response(h, p, wl.nocc))
                         for p in wl.H1.astype(np.float64)])
    np.testing.assert_allclose(r_dual, r_direct, rtol=1e-11)


def test_directional_fd_matches_dual_response():
    wl = W.dense_gapped(128)
    h = wl.H.astype(np.float64)
    a = wl.A[0].astype(np.float64)
    chi = cf.susceptibility(h, a, wl.nocc)
    for p in wl.H1[:3].astype(np.float64):
        g = fd.directional(h, a, wl.nocc, p, step=1e-4)
        assert abs(g - cf.response(chi, p)[0]) < 1e-7 * max(1.0, abs(g))


def test_trivial_occupations():
    h = W.dense_gapped(16).H.astype(np.float64)
    a = np.eye(16)
    np.testing.assert_array_equal(cf.density_matrix(h, 0), np.zeros((16, 16)))
    np.testing.assert_array_equal(cf.density_matrix(h, 16), np.eye(16))
    assert not cf.susceptibility(h, a, 0).any()
    assert not cf.susceptibility(h, a, 16).any()


def test_gapless_raises():
    h = W.gapless(12, 6)
    with pytest.raises(cf.GaplessError):
        cf.density_matrix(h, 6)
    with pytest.raises(cf.GaplessError):
        cf.susceptibility(h, np.eye(12), 6)


def test_batched_responses_equal_single():
    """The stacked form is the single-perturbation definition applied per matrix."""
    wl = W.dense_gapped(64, nocc=20)
    h = wl.H.astype(np.float64)
    ps = np.stack([wl.A[0], wl.H1[0], wl.H1[1]]).astype(np.float64)
    out = cf.first_order_responses(h, ps, wl.nocc)
    for k in range(3):
        np.testing.assert_allclose(out[k], cf.first_order_response(h, ps[k], wl.nocc), rtol=0, atol=1e-13)
