"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (relative Frobenius error against the closed form):
  FP32 products                    D <= 1e-5, chi <= 1e-5
  split-FP16 products (hi+lo, 11-bit terms on scaled operands: 22 bits
  per operand, the dropped lo*lo is 2^-22 relative)  D, chi <= 1e-5
  split-BF16 products (hi+mid+lo)  D <= 1e-4, chi <= 1e-4
  two-term split (hi+lo, the paper's Eq. MixPrecMult scheme) is held to 1e-4
  on the dense cases; on the banded cases with the site-position observable
  it misses it (3-4e-4: the large occupied-occupied blocks of that
  observable amplify the 2^-17 representation error of two BF16 terms) and
  those cases are skipped with that reason.
  Runs with the residual correction (opts.refine) are held to 1e-5.
Partial recursions (a fixed number of steps) are compared with the oracle's
FP64 recursion run on the sigma sequence and bounds the GPU chose; there the
only difference is FP32/BF16 rounding, bounded per step.
"""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf
from oracle import sp2

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_fp16": 1e-5, "split3_bf16": 1e-4, "split_bf16": 1e-4, "split3x_bf16": 1e-4}
PRECS = ["fp32", "split_fp16", "split3_bf16", "split3x_bf16", "split_bf16"]


def _tol(prec, case):
    if prec == "split_bf16" and case.startswith("band"):
        pytest.skip("two-term BF16 split on the site-position observable: chi 3-4e-4 (measured), above 1e-4")
    return TOL[prec]


def _dm():
    import paper_2409_17033_amd as dm
    dm.load()
    return dm


def _dev(x, gpu):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(gpu)


def _np(t):
    return t.detach().double().cpu().numpy()


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


def _case(name):
    if name == "c1":
        return W.dense_gapped(128)
    if name == "dense300":
        return W.dense_gapped(300, nocc=117, cfg=11)
    if name == "band1000":
        return W.banded_gapped(1000, nocc=500, cfg=12, cache=False)
    if name == "band2048":
        return W.banded_gapped(2048, cfg=2, cache=False)
    raise KeyError(name)


@pytest.mark.parametrize("case", ["c1", "dense300"])
@pytest.mark.parametrize("steps", [1, 5])
@pytest.mark.parametrize("prec", PRECS)
def test_partial_recursion_matches_fp64(gpu, case, steps, prec):
    """max_iter = k stops after k steps (NOT_CONVERGED); D = X_{k+1}, chi = s Y_{k+1}."""
    dm = _dm()
    wl = _case(case)
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    chi, D, _, info = dm.susceptibility(H, A, wl.nocc, precision=prec, bounds="gershgorin",
                                        max_iter=steps, min_iter=steps + 1, project=False,
                                        spin=1.0, raise_on_error=False)
    assert info["status"] == "DMPT_ERR_NOT_CONVERGED" and info["m"] == steps
    h = wl.H.astype(np.float64)
    assert abs(info["emin"] - sp2.gershgorin_bounds(h)[0]) < 1e-9
    xs, beta = sp2.sp2_sequence(h, info["sigma"], info["emin"], info["emax"])
    y = sp2.forward_sweep(xs, info["sigma"], beta, wl.A[0].astype(np.float64))
    tol = 6e-5 * steps if prec in ("split_bf16", "split3x_bf16") else 2e-6 * steps
    assert cf.rel_frobenius(_np(D), xs[-1]) < tol
    assert cf.rel_frobenius(_np(chi), y) < tol
    # the device traces are the FP64 traces of the stored iterates
    for n in range(steps + 1):
        assert abs(info["trace_x"][n] - np.trace(xs[n])) < 1e-4 * wl.n


@pytest.mark.parametrize("case", ["c1", "dense300", "band1000", "band2048"])
@pytest.mark.parametrize("prec", PRECS)
def test_converged_matches_closed_form(gpu, case, prec):
    tol = _tol(prec, case)
    dm = _dm()
    wl = _case(case)
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    chi, D, a0, info = dm.susceptibility(H, A, wl.nocc, precision=prec)
    h, a = wl.H.astype(np.float64), wl.A[0].astype(np.float64)
    dref = cf.density_matrix(h, wl.nocc)
    chiref = cf.susceptibility(h, a, wl.nocc, spin=2.0)
    ed, ec = cf.rel_frobenius(_np(D), dref), cf.rel_frobenius(_np(chi), chiref)
    print(f"{case} {prec}: M={info['m']} errD={ed:.2e} errchi={ec:.2e} {info['elapsed_ms']:.1f} ms")
    assert ed <= TOL[prec] and ec <= tol
    a0ref = 2.0 * cf.expectation(a, dref)
    assert abs(a0[0] - a0ref) <= TOL[prec] * max(1.0, np.abs(a).sum() / wl.n * wl.nocc)
    c = _np(chi)
    assert np.array_equal(c, c.T)                       # mirror store: exact symmetry
    assert abs(np.trace(c)) <= 10 * tol * np.linalg.norm(c) * np.sqrt(wl.n)


@pytest.mark.parametrize("case", ["c1", "dense300", "band1000"])
@pytest.mark.parametrize("prec", ["fp32", "split_fp16", "split3_bf16", "split3x_bf16"])
def test_refined_matches_closed_form(gpu, case, prec):
    """opts.refine: the residual correction after the projection brings chi to
    FP32 level (1e-5) for every precision whose D is FP32-accurate."""
    dm = _dm()
    wl = _case(case)
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    chi, D, a0, info = dm.susceptibility(H, A, wl.nocc, precision=prec, refine=True, profile=True)
    h, a = wl.H.astype(np.float64), wl.A[0].astype(np.float64)
    chiref = cf.susceptibility(h, a, wl.nocc, spin=2.0)
    ec = cf.rel_frobenius(_np(chi), chiref)
    print(f"{case} {prec} refined: M={info['m']} errchi={ec:.2e} refine {info['refine_ms']:.2f} ms")
    assert ec <= 1e-5
    c = _np(chi)
    assert abs(np.trace(c)) <= 1e-4 * np.linalg.norm(c) * np.sqrt(wl.n)


@pytest.mark.parametrize("case", ["c1", "dense300", "band1000"])
@pytest.mark.parametrize("prec", ["fp32", "split_fp16", "split3x_bf16"])
def test_sweep_tol_matches_closed_form(gpu, case, prec):
    """opts.sweep_tol with the residual correction: the sweep stops once X_n
    is within 1e-3 of idempotency and the correction's sweep within
    sqrt(1e-3); the correction removes the truncation error, so chi is held
    to the same 1e-5 as the full sweeps, and both sweeps must actually have
    stopped early."""
    dm = _dm()
    wl = _case(case)
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    chi, D, a0, info = dm.susceptibility(H, A, wl.nocc, precision=prec, refine=True, sweep_tol=1e-3)
    h, a = wl.H.astype(np.float64), wl.A[0].astype(np.float64)
    chiref = cf.susceptibility(h, a, wl.nocc, spin=2.0)
    ec = cf.rel_frobenius(_np(chi), chiref)
    ed = cf.rel_frobenius(_np(D), cf.density_matrix(h, wl.nocc))
    m = info["m"]
    print(f"{case} {prec} sweep_tol 1e-3: M={m} sweep {info['sweep_steps']} correction "
          f"{info['correction_steps']} errD={ed:.2e} errchi={ec:.2e}")
    assert ec <= 1e-5 and ed <= 1e-5
    assert info["sweep_steps"] < m and info["correction_steps"] < m
    eps = info["idem_x"]
    # the sweep kept Y_k for the first X_{k-1} within the tolerance
    k = info["sweep_steps"] + 1
    assert eps[k - 2] <= 1e-6 and all(e > 1e-6 for e in eps[:k - 2])
    assert eps[info["correction_steps"] - 1] <= 1e-3


def test_split_tail_tiles_match_closed_form(gpu):
    """N = 2048, split3x with the correction: the launches' lists end with
    K-split tiles (two half-K jobs each, added by a combine launch) where the
    makespan model picks them; chi must meet the refined 1e-5 against the
    closed form and agree with refine = 2 (regular tiles only, no split)
    to the accumulation-order level."""
    dm = _dm()
    wl = _case("band2048")
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    chi, D, _, info = dm.susceptibility(H, A, wl.nocc, precision="split3x_bf16", refine=1, sweep_tol=1e-3)
    chi2, _, _, info2 = dm.susceptibility(H, A, wl.nocc, precision="split3x_bf16", refine=2, sweep_tol=1e-3)
    h = wl.H.astype(np.float64)
    chiref = cf.susceptibility(h, wl.A[0].astype(np.float64), wl.nocc, spin=2.0)
    ec, ec2 = cf.rel_frobenius(_np(chi), chiref), cf.rel_frobenius(_np(chi2), chiref)
    print(f"split tiles {info['split_tiles']} (step), {info['split_tiles_sweep']} (sweep); errchi {ec:.2e}, "
          f"regular tiles {ec2:.2e}")
    assert info["split_tiles"] + info["split_tiles_sweep"] > 0
    assert info2["split_tiles"] == 0 and info2["split_tiles_sweep"] == 0
    assert ec <= 1e-5 and ec2 <= 1e-5
    assert cf.rel_frobenius(_np(chi), _np(chi2)) <= 5e-6
    assert cf.rel_frobenius(_np(D), cf.density_matrix(h, wl.nocc)) <= 1e-5


def test_headline_path_four_observables(gpu):
    """The timed configuration (split3x with the correction, sweep_tol 1e-3)
    on four random observables at N = 4096: one list of wide and regular
    sweep tiles for all four plus the X^2 tiles, with a K-split tail, in every
    step; each chi against its closed form at the refined 1e-5, and each
    equal to its single-observable run within that tolerance (the lists, and
    so the accumulation orders, differ; 3.6e-6 measured)."""
    dm = _dm()
    wl = W.banded_gapped(4096, observable="random", nobs=4, npert=1, cfg=15, cache=False)
    H, A = _dev(wl.H, gpu), _dev(wl.A, gpu)
    kw = dict(precision="split3x_bf16", refine=True, sweep_tol=1e-3)
    chi, D, _, info = dm.susceptibility(H, A, wl.nocc, **kw)
    h = wl.H.astype(np.float64)
    refs = 2.0 * cf.first_order_responses(h, wl.A.astype(np.float64), wl.nocc)
    print(f"M={info['m']} sweep {info['sweep_steps']} correction {info['correction_steps']} "
          f"split tiles {info['split_tiles']} / {info['split_tiles_sweep']}")
    assert info["split_tiles"] > 0 and info["sweep_steps"] < info["m"]
    assert cf.rel_frobenius(_np(D), cf.density_matrix(h, wl.nocc)) <= 1e-5
    for k, ref in enumerate(refs):
        ek = cf.rel_frobenius(_np(chi[k]), ref)
        one, _, _, _ = dm.susceptibility(H, A[k].contiguous(), wl.nocc, **kw)
        e1 = cf.rel_frobenius(_np(one), _np(chi[k]))
        print(f"obs {k}: errchi {ek:.2e}, single run differs by {e1:.2e}")
        assert ek <= 1e-5 and e1 <= 1e-5


def test_accurate_projections_three_observables(gpu):
    """project = 2 (Y projected in three terms, the correction's delta in two)
    with the timed configuration on three random observables at N = 2048:
    each chi against its closed form at the refined 1e-5, each equal to its
    single-observable run, and D untouched by the option (bit for bit)."""
    dm = _dm()
    wl = W.banded_gapped(2048, observable="random", nobs=3, npert=1, cfg=16, cache=False)
    H, A = _dev(wl.H, gpu), _dev(wl.A, gpu)
    kw = dict(precision="split3x_bf16", refine=True, sweep_tol=1e-3)
    chi, D, _, info = dm.susceptibility(H, A, wl.nocc, project=2, **kw)
    chi1, D1, _, _ = dm.susceptibility(H, A, wl.nocc, **kw)
    refs = 2.0 * cf.first_order_responses(wl.H.astype(np.float64), wl.A.astype(np.float64), wl.nocc)
    assert torch_equal(D, D1)
    for k, ref in enumerate(refs):
        e2 = cf.rel_frobenius(_np(chi[k]), ref)
        e1 = cf.rel_frobenius(_np(chi1[k]), ref)
        one, _, _, _ = dm.susceptibility(H, A[k].contiguous(), wl.nocc, project=2, **kw)
        d1 = cf.rel_frobenius(_np(one), _np(chi[k]))
        print(f"obs {k}: errchi project=2 {e2:.2e} (project=1 {e1:.2e}), single run differs by {d1:.2e}")
        assert e2 <= 1e-5 and d1 <= 1e-5


def test_refine_two_observables(gpu):
    """The correction runs every observable through one BF16 sweep: each must
    match its own closed form, and the batch must equal the single runs."""
    dm = _dm()
    wl = W.dense_gapped(300, nocc=117, nobs=2, cfg=13)
    H, A = _dev(wl.H, gpu), _dev(wl.A, gpu)
    chi, _, _, _ = dm.susceptibility(H, A, wl.nocc, precision="split_fp16", refine=True)
    h = wl.H.astype(np.float64)
    for k in range(2):
        ref = cf.susceptibility(h, wl.A[k].astype(np.float64), wl.nocc, 2.0)
        assert cf.rel_frobenius(_np(chi[k]), ref) <= 1e-5
        one, _, _, _ = dm.susceptibility(H, A[k].contiguous(), wl.nocc, precision="split_fp16", refine=True)
        assert cf.rel_frobenius(_np(one), _np(chi[k])) <= 1e-6


def test_refined_wide_and_regular_tiles(gpu):
    """split3x_bf16 with the correction at N = 2000 (padded to 2048), eight
    random observables: the steps run their sweep products on 256 x 256 tiles
    only, the projection and correction launches on a list of both kinds (72
    wide and 432 regular tiles on 256 CUs), and refine = 2 runs everything on
    the regular tiles.  Each observable is held to 1e-5 against the closed
    form in both runs; the runs differ in accumulation order only."""
    dm = _dm()
    wl = W.banded_gapped(2000, nocc=1000, observable="random", nobs=8, npert=1, cfg=14, cache=False)
    H, A = _dev(wl.H, gpu), _dev(wl.A, gpu)
    chi_w, _, _, info_w = dm.susceptibility(H, A, wl.nocc, precision="split3x_bf16", refine=1, profile=True)
    chi_r, _, _, info_r = dm.susceptibility(H, A, wl.nocc, precision="split3x_bf16", refine=2, profile=True)
    refs = 2.0 * cf.first_order_responses(wl.H.astype(np.float64), wl.A.astype(np.float64), wl.nocc)
    for k, ref in enumerate(refs):
        ew = cf.rel_frobenius(_np(chi_w[k]), ref)
        er = cf.rel_frobenius(_np(chi_r[k]), ref)
        print(f"obs {k}: wide {ew:.2e} regular {er:.2e}")
        assert ew <= 1e-5 and er <= 1e-5
        assert cf.rel_frobenius(_np(chi_w[k]), _np(chi_r[k])) <= 5e-6
    print(f"wide: steps {info_w['step_ms']:.2f} ms refine {info_w['refine_ms']:.2f} ms; "
          f"regular: steps {info_r['step_ms']:.2f} ms refine {info_r['refine_ms']:.2f} ms")


@pytest.mark.parametrize("prec", PRECS)
def test_sp2_density(gpu, prec):
    dm = _dm()
    wl = _case("band1000")
    D, info = dm.sp2_density(_dev(wl.H, gpu), wl.nocc, precision=prec)
    dref = cf.density_matrix(wl.H.astype(np.float64), wl.nocc)
    assert cf.rel_frobenius(_np(D), dref) <= TOL[prec]
    assert abs(info["trace_d"] - wl.nocc) < TOL[prec] * wl.nocc
    d = _np(D)
    assert abs(np.trace(d) - info["trace_d"]) < 1e-3


def test_duality_on_gpu(gpu):
    """Tr[chi^A H1] = s Tr[A D1] with D1 from the same kernels (A := H1, s = 1)."""
    dm = _dm()
    wl = _case("c1")
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    H1 = _dev(wl.H1, gpu)
    chi, _, _, _ = dm.susceptibility(H, A, wl.nocc)
    dual = dm.response(chi, H1)[0]
    d1, _, _, _ = dm.susceptibility(H, H1, wl.nocc, spin=1.0)   # 8 observables = 8 D1
    direct = 2.0 * dm.response(d1, A.unsqueeze(0).contiguous())[:, 0]
    ref = cf.response(cf.susceptibility(wl.H.astype(np.float64), wl.A[0].astype(np.float64),
                                        wl.nocc, 2.0), wl.H1)
    scale = np.abs(ref).max()
    assert np.max(np.abs(dual - ref)) <= 1e-5 * scale
    assert np.max(np.abs(direct - ref)) <= 1e-5 * scale


def test_response_kernel(gpu):
    dm = _dm()
    rng = np.random.default_rng(3)
    for n, k, p in [(1, 1, 1), (37, 2, 3), (300, 1, 8), (513, 3, 11)]:
        chi = rng.normal(size=(k, n, n)).astype(np.float32)
        h1 = rng.normal(size=(p, n, n)).astype(np.float32)
        out = dm.response(_dev(chi, gpu), _dev(h1, gpu))
        ref = np.einsum("kij,pij->kp", chi.astype(np.float64), h1.astype(np.float64))
        assert np.allclose(out, ref, rtol=1e-12, atol=1e-9 * n)


@pytest.mark.parametrize("prec", ["fp32", "split_fp16", "split3_bf16"])
def test_projection_after_either_last_sigma(gpu, prec):
    """The launch after the last step runs before the stop is seen; when it
    took sigma = +1 its Y is the first projection step, which is then not
    launched again.  Seeded systems with both values of that sigma must match
    the closed form (info["sigma_next"] reports it)."""
    dm = _dm()
    seen = set()
    for seed in range(12):
        n, nocc = 200, 60 + 7 * seed
        h, _, _ = W.known_spectrum(n, nocc, gap=0.3, seed=seed)
        a = W.random_perturbations(n, 2, seed=100 + seed)      # two observables: one pass each
        h32, a32 = h.astype(np.float32), a.astype(np.float32)
        chi, D, a0, info = dm.susceptibility(_dev(h32, gpu), _dev(a32, gpu), nocc, precision=prec)
        seen.add(info["sigma_next"])
        for k in range(2):
            ref = cf.susceptibility(h32.astype(np.float64), a32[k].astype(np.float64), nocc, spin=2.0)
            err = cf.rel_frobenius(_np(chi[k]), ref)
            print(f"seed {seed} nocc {nocc} obs {k} {prec}: M={info['m']} sigma_next={info['sigma_next']} "
                  f"errchi={err:.2e}")
            assert err <= TOL[prec], (seed, k)
    assert seen == {1, -1}, seen


@pytest.mark.parametrize("prec", PRECS)
def test_adjoint_sweep_matches_forward(gpu, prec):
    dm = _dm()
    wl = _case("dense300")
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    chi_f, _, _, inf_f = dm.susceptibility(H, A, wl.nocc, precision=prec)
    chi_b, _, _, inf_b = dm.susceptibility(H, A, wl.nocc, precision=prec, sweep="adjoint")
    ref = cf.susceptibility(wl.H.astype(np.float64), wl.A[0].astype(np.float64), wl.nocc, 2.0)
    assert cf.rel_frobenius(_np(chi_b), ref) <= TOL[prec]
    assert cf.rel_frobenius(_np(chi_b), _np(chi_f)) <= 2 * TOL[prec]


def test_multiple_observables(gpu):
    dm = _dm()
    wl = W.dense_gapped(200, nocc=90, nobs=3, cfg=13)
    chi, _, a0, _ = dm.susceptibility(_dev(wl.H, gpu), _dev(wl.A, gpu), wl.nocc)
    h = wl.H.astype(np.float64)
    for k in range(3):
        ref = cf.susceptibility(h, wl.A[k].astype(np.float64), wl.nocc, 2.0)
        assert cf.rel_frobenius(_np(chi[k]), ref) <= 1e-5


def test_trivial_occupations(gpu):
    dm = _dm()
    wl = _case("c1")
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    chi, D, a0, _ = dm.susceptibility(H, A, 0)
    assert not _np(D).any() and not _np(chi).any() and a0[0] == 0.0
    chi, D, a0, _ = dm.susceptibility(H, A, wl.n)
    assert np.array_equal(_np(D), np.eye(wl.n)) and not _np(chi).any()
    assert abs(a0[0] - 2.0 * np.trace(wl.A[0].astype(np.float64))) < 1e-9 * wl.n


def test_tiny_matrices(gpu):
    dm = _dm()
    g = {"H": [[0.0, 1.0], [1.0, 0.0]], "A": [[1.0, 0.0], [0.0, -1.0]]}
    chi, D, _, _ = dm.susceptibility(_dev(g["H"], gpu), _dev(g["A"], gpu), 1, spin=1.0)
    assert np.allclose(_np(D), [[0.5, -0.5], [-0.5, 0.5]], atol=1e-6)
    assert np.allclose(_np(chi), [[-0.5, 0.0], [0.0, 0.5]], atol=1e-5)
    D1, _ = dm.sp2_density(_dev([[0.3]], gpu), 1)
    assert abs(_np(D1)[0, 0] - 1.0) < 1e-6


@pytest.mark.parametrize("n", [3, 17, 129, 257])
@pytest.mark.parametrize("prec", PRECS)
def test_ragged_sizes(gpu, n, prec):
    """Sizes that leave a ragged tail in the 256-padded tiles (and tiny ones)."""
    dm = _dm()
    nocc = max(1, n // 3)
    h, _, _ = W.known_spectrum(n, nocc, gap=0.3, seed=n)
    a = W.random_perturbations(n, 1, seed=n)[0] * n
    h32, a32 = h.astype(np.float32), a.astype(np.float32)
    chi, D, a0, info = dm.susceptibility(_dev(h32, gpu), _dev(a32, gpu), nocc, precision=prec)
    h64, a64 = h32.astype(np.float64), a32.astype(np.float64)
    dref = cf.density_matrix(h64, nocc)
    chiref = cf.susceptibility(h64, a64, nocc, spin=2.0)
    assert cf.rel_frobenius(_np(D), dref) <= TOL[prec]
    assert cf.rel_frobenius(_np(chi), chiref) <= TOL[prec]
    assert abs(a0[0] - 2.0 * cf.expectation(a64, dref)) <= 2 * TOL[prec] * np.linalg.norm(a64) * np.linalg.norm(dref)


def test_error_statuses(gpu):
    dm = _dm()
    wl = _case("c1")
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    bad = wl.H.copy()
    bad[3, 5] = np.nan
    with pytest.raises(dm.DMPTError) as e:
        dm.susceptibility(_dev(bad, gpu), A, wl.nocc)
    assert e.value.status_name == "DMPT_ERR_NONFINITE"
    w = np.linalg.eigvalsh(wl.H.astype(np.float64))
    with pytest.raises(dm.DMPTError) as e:
        dm.susceptibility(H, A, wl.nocc, bounds="given", emin=0.5 * (w[0] + w[-1]), emax=w[-1] + 0.1)
    assert e.value.status_name == "DMPT_ERR_BOUNDS"
    with pytest.raises(dm.DMPTError) as e:
        dm.susceptibility(H, A, wl.nocc, max_iter=3)
    assert e.value.status_name == "DMPT_ERR_NOT_CONVERGED"
    # no gap: the degenerate pair stays near x = 1/2 (eps_n ~ 0.12 >= 1/64) until
    # FP32 rounding splits it (~90 steps in an FP32 emulation); 40 steps are ample
    # for any gapped case here.
    gl = W.gapless(128, 64).astype(np.float32)
    with pytest.raises(dm.DMPTError) as e:
        dm.sp2_density(_dev(gl, gpu), 64, max_iter=40)
    assert e.value.status_name == "DMPT_ERR_NOT_CONVERGED"


def test_deterministic(gpu):
    dm = _dm()
    wl = _case("dense300")
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    c1, d1, _, i1 = dm.susceptibility(H, A, wl.nocc, precision="split3_bf16")
    c2, d2, _, i2 = dm.susceptibility(H, A, wl.nocc, precision="split3_bf16")
    assert i1["sigma"] == i2["sigma"]
    assert np.array_equal(_np(c1), _np(c2)) and np.array_equal(_np(d1), _np(d2))
