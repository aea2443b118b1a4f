"""Pins for the FP64 SP2 / susceptibility recursion oracle (CPU only)."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf
from oracle import sp2


@pytest.fixture(scope="module")
def c1():
    wl = W.dense_gapped(128)
    return wl.H.astype(np.float64), wl.A[0].astype(np.float64), wl.H1.astype(np.float64), wl.nocc


def test_gershgorin_encloses_spectrum(c1):
    h = c1[0]
    lo, hi = sp2.gershgorin_bounds(h)
    w = np.linalg.eigvalsh(h)
    assert lo <= w[0] and w[-1] <= hi


def test_gershgorin_hand_worked_discs():
    """Disc endpoints worked by hand (all dyadic, so exact in FP64).
    Rows of h: centre 2, radius 1.5 -> [0.5, 3.5]; centre 0, radius 1.25 ->
    [-1.25, 1.25]; centre -3, radius 0.75 -> [-3.75, -2.25].  The interval is
    the union's hull [-3.75, 3.5]; a radius that also counted the diagonal,
    or missed the absolute value, gives another interval."""
    h = np.array([[2.0, -1.0, 0.5], [-1.0, 0.0, 0.25], [0.5, 0.25, -3.0]])
    assert sp2.gershgorin_bounds(h) == (-3.75, 3.5)
    # [[1, 1], [1, 1]]: both discs are [0, 2], which is exactly the spectrum {0, 2}
    assert sp2.gershgorin_bounds(np.ones((2, 2))) == (0.0, 2.0)
    # a diagonal matrix: radius 0, the bounds are its extreme entries
    assert sp2.gershgorin_bounds(np.diag([0.3, -1.5, 4.0])) == (-1.5, 4.0)


def test_sigma_rule_picks_closest_trace():
    rng = np.random.default_rng(1)
    for _ in range(20):
        q, _ = np.linalg.qr(rng.normal(size=(12, 12)))
        x = (q * rng.uniform(0, 1, 12)) @ q.T
        nocc = int(rng.integers(1, 12))
        t_sq = np.trace(x @ x)
        t_ot = np.trace(2 * x - x @ x)
        want = 1 if abs(t_sq - nocc) <= abs(t_ot - nocc) else -1
        assert sp2.choose_sigma(np.trace(x), np.sum(x * x), nocc) == want


def test_diagonal_h_gives_exact_step_function():
    e = np.array([0.7, -1.2, 0.1, 2.0, -0.3, 1.1, -2.0, 0.4])
    nocc = 3
    d, tr = sp2.sp2_density(np.diag(e), nocc)
    want = np.zeros(8)
    want[np.argsort(e)[:nocc]] = 1.0
    np.testing.assert_allclose(d, np.diag(want), atol=1e-12)
    assert tr.m >= 10
    # on a diagonal H every step acts on each eigenvalue alone: the recorded
    # sigma sequence, applied to the scalars x_i = (emax - e_i) / (emax - emin),
    # must give the same step function
    x = (tr.emax - e) / (tr.emax - tr.emin)
    for s in tr.sigmas:
        x = x * x if s > 0 else 2 * x - x * x
    np.testing.assert_allclose(x, want, atol=1e-12)


def test_diagonal_h_susceptibility_is_textbook():
    rng = np.random.default_rng(4)
    e = rng.permutation(np.linspace(-1.5, 1.5, 10))
    a = rng.normal(size=(10, 10))
    a = a + a.T
    _, chi, _, _ = sp2.sp2_susceptibility(np.diag(e), a, 4)
    occ, vir = np.argsort(e)[:4], np.argsort(e)[4:]
    ref = np.zeros((10, 10))
    for i in occ:
        for v in vir:
            ref[i, v] = ref[v, i] = a[i, v] / (e[i] - e[v])
    np.testing.assert_allclose(chi, ref, atol=1e-10)


def test_converged_recursion_matches_closed_form(c1):
    h, a, _, nocc = c1
    d, chi, a0, tr = sp2.sp2_susceptibility(h, a, nocc, spin=2.0)
    assert cf.rel_frobenius(d, cf.density_matrix(h, nocc)) < 1e-11
    assert cf.rel_frobenius(chi, cf.susceptibility(h, a, nocc, spin=2.0)) < 1e-10
    assert abs(a0 - 2 * cf.expectation(a, cf.density_matrix(h, nocc))) < 1e-10 * max(1, abs(a0))
    assert 10 <= tr.m < 100


def test_known_spectrum_density(c1):
    h, w, q = W.known_spectrum(96, 40, gap=0.2, seed=7)
    d, _ = sp2.sp2_density(h, 40)
    np.testing.assert_allclose(d, q[:, :40] @ q[:, :40].T, atol=1e-11)


def test_duality_exact_for_unconverged_recursion(c1):
    """Tr[A Y^{H1}_{M+1}] = Tr[H1 Y^{A}_{M+1}] holds for any fixed sigma sequence."""
    h, a, h1s, nocc = c1
    emin, emax = sp2.gershgorin_bounds(h)
    sig = [1, -1, -1, 1, -1]
    xs, beta = sp2.sp2_sequence(h, sig, emin, emax)
    y_a = sp2.forward_sweep(xs, sig, beta, a)
    for p in h1s[:4]:
        y_p = sp2.forward_sweep(xs, sig, beta, p)
        lhs, rhs = np.sum(a * y_p), np.sum(p * y_a)
        assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1e-300) + 1e-15


def test_forward_equals_backward_unconverged(c1):
    """Eq. (DM2) and Eq. (DM3) give the same chi for any fixed sequence."""
    h, a, _, _ = c1
    emin, emax = sp2.gershgorin_bounds(h)
    sig = [1, -1, -1, 1, -1, 1, 1, -1]
    xs, beta = sp2.sp2_sequence(h, sig, emin, emax)
    fwd = sp2.forward_sweep(xs, sig, beta, a)
    bwd = sp2.backward_sweep(xs, sig, beta, a)
    assert cf.rel_frobenius(bwd, fwd) < 1e-12


def test_backward_converged_matches_closed_form(c1):
    h, a, _, nocc = c1
    _, chi, _ = sp2.sp2_backward_susceptibility(h, a, nocc, spin=2.0)
    assert cf.rel_frobenius(chi, cf.susceptibility(h, a, nocc, spin=2.0)) < 1e-10


def test_recursion_derivative_equals_fd_of_recursion(c1):
    """chi from Eq. (DM3) is the exact derivative of Tr[A X_{M+1}(H)] for fixed sigma."""
    h, a, h1s, nocc = c1
    emin, emax = sp2.gershgorin_bounds(h)
    sig = [1, -1, -1, 1, -1, 1, -1, 1, 1, -1]
    xs, beta = sp2.sp2_sequence(h, sig, emin, emax)
    chi = sp2.forward_sweep(xs, sig, beta, a)
    for p in h1s[:3]:
        step = 1e-4
        fp = np.sum(a * sp2.sp2_sequence(h + step * p, sig, emin, emax)[0][-1])
        fm = np.sum(a * sp2.sp2_sequence(h - step * p, sig, emin, emax)[0][-1])
        g = (fp - fm) / (2 * step)
        assert abs(g - np.sum(chi * p)) < 1e-8 * max(1.0, abs(g))


def test_dmpert_duality_converged(c1):
    """Eq. (DMPert) vs Eq. (DMSuscept): s Tr[A D1] = Tr[chi H1] (s = 2)."""
    h, a, h1s, nocc = c1
    _, chi, _, _ = sp2.sp2_susceptibility(h, a, nocc, spin=2.0)
    for p in h1s:
        _, d1, _ = sp2.sp2_density_response(h, p, nocc)
        assert abs(2 * np.sum(a * d1) - np.sum(chi * p)) < 1e-11 * abs(np.sum(chi * p))


def test_bounds_not_enclosing_raises(c1):
    h, a, _, nocc = c1
    w = np.linalg.eigvalsh(h)
    with pytest.raises(sp2.BoundsError):
        sp2.sp2_susceptibility(h, a, nocc, emin=w[0] + 0.5 * (w[-1] - w[0]), emax=w[-1])


def test_gapless_not_converged():
    """Without a gap a state stays near x = 1/2 (eps >= 1/64), so the stopping
    test never fires; only rounding, ~log2(width / 1e-16) steps later, would
    split the degenerate pair.  A 40-step limit (ample for any real gap)
    reports it."""
    h = W.gapless(24, 12)
    with pytest.raises(sp2.NotConvergedError):
        sp2.sp2_density(h, 12, max_iter=40)


def test_stop_is_at_rounding_floor():
    """The idempotency error at the stop is at the FP64 floor, far below the
    unresolved threshold, and the stop fired on stagnation or the tolerance."""
    wl = W.dense_gapped(128)
    _, tr = sp2.sp2_density(wl.H.astype(np.float64), wl.nocc)
    assert tr.errors[-1] < 1e-20
    assert tr.errors[-1] >= tr.errors[-3] or tr.errors[-1] == 0.0


def test_max_iter_not_converged(c1):
    h, a, _, nocc = c1
    with pytest.raises(sp2.NotConvergedError):
        sp2.sp2_susceptibility(h, a, nocc, max_iter=3)


def test_trivial_occupations(c1):
    h, a, _, _ = c1
    d, chi, a0, _ = sp2.sp2_susceptibility(h, a, 0)
    assert not d.any() and not chi.any() and a0 == 0
    d, chi, a0, _ = sp2.sp2_susceptibility(h, a, 128)
    np.testing.assert_array_equal(d, np.eye(128))
    assert not chi.any()
