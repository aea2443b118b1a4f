"""Pins for the self-consistent response oracle (Eq. CP_SCF / DM_CP_SCF) and
the mixer-network oracle (CPU only)."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf
from oracle import mlp
from oracle import scf


def _system(n, nocc, seed):
    h, _, _ = W.known_spectrum(n, nocc, gap=0.4, seed=seed)
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.5, 1.5, size=n)
    a = W.random_perturbations(n, 1, seed=seed + 1)[0]
    h1 = np.diag(rng.normal(0.0, 0.01, size=n))
    return h, u, a, h1


def test_no_interaction_is_plain_susceptibility():
    h, u, a, _ = _system(24, 9, 3)
    chi, it, _ = scf.scf_susceptibility(h, a, 0.0 * u, 9, spin=2.0, mix=1.0)
    np.testing.assert_allclose(chi, cf.susceptibility(h, a, 9, spin=2.0), atol=1e-14)
    assert it <= 2


def test_duality_self_consistent():
    """Tr[chi H1] = s Tr[A D1] with both sides self-consistent (Table 1's
    comparison, here on a synthetic system)."""
    h, u, a, h1 = _system(48, 20, 5)
    chi, _, _ = scf.scf_susceptibility(h, a, u, 20, spin=2.0)
    d1, _, _ = scf.scf_density_response(h, h1, u, 20, spin=2.0)
    lhs, rhs = float(np.sum(chi * h1)), 2.0 * float(np.sum(a * d1))
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1e-300)
    # the interaction matters: the non-self-consistent answer differs
    assert abs(lhs - float(np.sum(cf.susceptibility(h, a, 20, 2.0) * h1))) > 1e-6 * abs(lhs)


def test_iteration_reaches_affine_fixed_point():
    h, u, a, _ = _system(16, 6, 7)
    chi, _, _ = scf.scf_susceptibility(h, a, u, 6, spin=2.0)
    f0, jac, vstar = scf.scf_fixed_point_map(h, a, u, 6, spin=2.0)
    np.testing.assert_allclose(np.diag(chi) / 2.0, vstar, atol=1e-12)
    # chi' = L[A + G(chi')] holds for the whole matrix, not only its diagonal
    lmap = scf.FirstOrder(h, 6)
    np.testing.assert_allclose(chi / 2.0, lmap(a + scf.onsite_field(chi / 2.0, u, 2.0)), atol=1e-12)


def test_finite_difference_of_scf_ground_state():
    """chi is the derivative of <A> = s Tr[A D] of the self-consistent ground
    state of H0 + lambda H1 (brute force, tiny n)."""
    n, nocc = 10, 4
    h, u, a, _ = _system(n, nocc, 11)
    h1 = W.random_perturbations(n, 1, seed=12)[0]
    chi, _, _ = scf.scf_susceptibility(h, a, u, nocc, spin=2.0)
    step = 1e-5
    dp = scf.scf_ground_state(h, u, nocc, 2.0, h_ext=step * h1)
    dm = scf.scf_ground_state(h, u, nocc, 2.0, h_ext=-step * h1)
    fd = 2.0 * float(np.sum(a * (dp - dm))) / (2 * step)
    assert abs(fd - float(np.sum(chi * h1))) <= 1e-7 * max(1.0, abs(fd))


def test_ground_state_without_field_is_d_of_h0():
    h, u, _, _ = _system(12, 5, 13)
    np.testing.assert_allclose(scf.scf_ground_state(h, u, 5), cf.density_matrix(h, 5), atol=1e-13)


# ------------------------------------------------------------------ mixer network

def test_mlp_site_inputs_by_hand():
    """n = 3, window 1: site i sees (x_{i-1}, x_i, x_{i+1}, e_{i-1}, e_i, e_{i+1}, U_i),
    zeros off the ends."""
    z = mlp.site_inputs(np.array([[1.0, 2.0, 3.0]]), np.array([0.5, 0.6, 0.7]), np.array([-1.0, 0.25, 2.0]), 1)
    np.testing.assert_array_equal(z, [[0, 1, 2, 0, -1.0, 0.25, 0.5],
                                      [1, 2, 3, -1.0, 0.25, 2.0, 0.6],
                                      [2, 3, 0, 0.25, 2.0, 0, 0.7]])


def test_mlp_site_inputs_wide_window_brute_force():
    """A window wider than the system (w = 5, n = 3) and a ragged case, against
    the definition entry by entry: z[(b, i), d + w] = x_b,i+d and
    z[(b, i), 2w + 1 + d + w] = e_i+d inside, 0 outside."""
    rng = np.random.default_rng(4)
    for n, w in ((3, 5), (6, 2), (1, 0)):
        x, u, e = rng.normal(size=(2, n)), rng.uniform(0.5, 1.5, size=n), rng.uniform(-1, 1, size=n)
        z = mlp.site_inputs(x, u, e, w)
        assert z.shape == (2 * n, 4 * w + 3)
        for b in range(2):
            for i in range(n):
                row = z[b * n + i]
                for d in range(-w, w + 1):
                    inside = 0 <= i + d < n
                    assert row[d + w] == (x[b, i + d] if inside else 0.0)
                    assert row[2 * w + 1 + d + w] == (e[i + d] if inside else 0.0)
                assert row[-1] == u[i]


def test_mlp_hand_example():
    """window 0, h = 1: y_i = w2 tanh(w1 . (x_i, e_i, U_i) + b1) + b2."""
    p = np.array([0.7, 0.3, -0.4, -0.2, 1.5, 0.1])   # W1 = [0.7, 0.3, -0.4], b1, w2, b2
    y, _, _ = mlp.forward(p, np.array([[0.3, -1.0]]), np.array([1.2, 0.8]), np.array([0.5, -2.0]), 0, 1)
    want = [1.5 * np.tanh(0.7 * 0.3 + 0.3 * 0.5 - 0.4 * 1.2 - 0.2) + 0.1,
            1.5 * np.tanh(-0.7 - 0.6 - 0.4 * 0.8 - 0.2) + 0.1]
    np.testing.assert_allclose(y[0], want, rtol=1e-15)


def test_mlp_gradient_matches_finite_differences():
    n, w, h, b = 7, 2, 4, 3
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.5, size=mlp.param_count(w, h))
    x = rng.normal(size=(b, n))
    t = rng.normal(size=(b, n))
    u = rng.uniform(0.5, 1.5, size=n)
    e = rng.uniform(-1, 1, size=n)
    _, g = mlp.loss_grad(p, x, t, u, e, w, h)
    step = 1e-6
    for i in range(p.size):
        d = np.zeros_like(p)
        d[i] = step
        fd = (mlp.loss_grad(p + d, x, t, u, e, w, h)[0] - mlp.loss_grad(p - d, x, t, u, e, w, h)[0]) / (2 * step)
        assert abs(fd - g[i]) <= 1e-8 * max(1.0, abs(fd)), i


def test_adam_first_step_closed_form():
    """Step 1: bias-corrected m = g and v = g^2, so p1 = p - lr g / (|g| + eps)."""
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
