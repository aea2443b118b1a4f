"""GPU parity on the water-cluster-shaped cases of Sec. VI (Table 2): 100
molecules, N = 2400 (ragged: padded to 2560), N_occ = 500 (about a fifth
filled, unlike the half-filled configs), and the largest, 301 molecules,
N = 7224 (padded to 7424), N_occ = 1505; gap 2 % of the spectral width,
A = site position, H1 = one random potential shift per atom.

Both routes of the duality (Fig. 1, Eqs. direct and dual) run on the GPU:
the susceptibility route Tr[chi^A H1] and the density-matrix-perturbation
route s Tr[A D1], with D1 computed by the same recursion with H1 in place
of A and s = 1.  The FP64 oracle is the Daleckii-Krein closed form.

Tolerances (relative Frobenius of chi, D and D1; response errors relative to
||chi||_F ||H1||_F, which bounds them by Cauchy-Schwarz): 1e-5 for FP32 and
the scaled FP16 split, 1e-4 for the three-term BF16 split at N = 2400; at
N = 7224 1e-5 for FP32 (its products sum their K-chunks in FP64) and the
1e-4 of split products for the FP16 split (measured there: 1.0e-5).
"""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "split_fp16": 1e-5, "split3_bf16": 1e-4, "split3x_bf16+refine@1e-3": 1e-5}
HEADLINE = "split3x_bf16+refine@1e-3"   # bench.py's default path


def _kw(path):
    """precision[+refine[@sweep_tol]] -> susceptibility() keywords."""
    prec, _, rest = path.partition("+")
    kw = {"precision": prec}
    if rest:
        kw["refine"] = True
        if "@" in rest:
            kw["sweep_tol"] = float(rest.partition("@")[2])
    return kw


@pytest.fixture(scope="module")
def water100():
    wl = W.water_shaped(100, cache=False)
    h = wl.H.astype(np.float64)
    a = wl.A[0].astype(np.float64)
    h1 = wl.H1[0].astype(np.float64)
    d = cf.density_matrix(h, wl.nocc)
    chi = cf.susceptibility(h, a, wl.nocc, spin=2.0)
    d1 = cf.density_response(h, h1, wl.nocc)
    return wl, d, chi, d1


@pytest.mark.parametrize("prec", ["fp32", "split_fp16", "split3_bf16", HEADLINE])
def test_water_shape_both_routes(gpu, water100, prec):
    import torch

    import paper_2409_17033_amd as dm
    wl, dref, chiref, d1ref = water100
    assert (wl.n, wl.nocc) == (2400, 500)
    H = torch.from_numpy(wl.H).to(gpu)
    A = torch.from_numpy(wl.A[0]).to(gpu)
    H1 = torch.from_numpy(wl.H1[0]).to(gpu)
    chi, D, a0, info = dm.susceptibility(H, A, wl.nocc, profile=True, **_kw(prec))
    d1, _, _, info1 = dm.susceptibility(H, H1, wl.nocc, spin=1.0, want_density=False, **_kw(prec))
    ed = cf.rel_frobenius(D.double().cpu().numpy(), dref)
    ec = cf.rel_frobenius(chi.double().cpu().numpy(), chiref)
    ed1 = cf.rel_frobenius(d1.double().cpu().numpy(), d1ref)
    r_chi = dm.response(chi, H1)[0, 0]                 # Tr[chi^A H1]
    r_d1 = 2.0 * dm.response(d1, A)[0, 0]              # s Tr[A D1]
    h1 = wl.H1[0].astype(np.float64)
    a64 = wl.A[0].astype(np.float64)
    rref = float(np.sum(chiref * h1))
    scale_chi = np.linalg.norm(chiref) * np.linalg.norm(h1)
    scale_d1 = 2.0 * np.linalg.norm(a64) * np.linalg.norm(d1ref)
    print(f"\nwater N=2400 {prec}: M={info['m']} (D1 route M={info1['m']}) errD={ed:.2e} errchi={ec:.2e} "
          f"errD1={ed1:.2e} Tr[chi H1]={r_chi:.8f} 2Tr[A D1]={r_d1:.8f} ref={rref:.8f}")
    tol = TOL[prec]
    assert ed <= tol and ec <= tol and ed1 <= tol
    assert abs(r_chi - rref) <= tol * scale_chi
    assert abs(r_d1 - rref) <= tol * scale_d1
    # the oracle's duality itself: s Tr[A D1] = Tr[chi^A H1] in FP64
    assert abs(2.0 * float(np.sum(a64 * d1ref)) - rref) <= 1e-10 * scale_chi


@pytest.fixture(scope="module")
def water301():
    import time
    wl = W.water_shaped(301, cache=False)
    t = time.perf_counter()
    h1 = wl.H1[0].astype(np.float64)
    # chi' of A and D1 of H1 from one eigendecomposition
    resp = cf.first_order_responses(wl.H.astype(np.float64), np.stack([wl.A[0].astype(np.float64), h1]), wl.nocc)
    chi, d1 = 2.0 * resp[0], resp[1]
    rref = float(np.sum(chi * h1))
    print(f"\nwater N=7224 closed form in {time.perf_counter() - t:.1f} s: Tr[chi H1] = {rref:.6f}", flush=True)
    return wl, chi, d1, rref, np.linalg.norm(chi) * np.linalg.norm(h1)


TOL_WATER = {"fp32": 1e-5, "split_fp16": 1e-4, HEADLINE: 1e-5}


@pytest.mark.parametrize("prec", ["fp32", "split_fp16", HEADLINE])
def test_water_shape_largest(gpu, water301, prec):
    """The largest shape of Table 2 (301 molecules, N = 7224, padded to 7424)
    in the launch configuration bench.py's shapes run times: chi against the
    closed form, and the chi route's response within the Cauchy-Schwarz bound
    the chi tolerance gives, tol ||chi||_F ||H1||_F; the D1 route is held to
    the same bound (by duality both estimate the same number)."""
    import torch

    import paper_2409_17033_amd as dm
    wl, chiref, d1ref, rref, scale = water301
    assert (wl.n, wl.nocc) == (7224, 1505)
    H = torch.from_numpy(wl.H).to(gpu)
    A = torch.from_numpy(wl.A[0]).to(gpu)
    H1 = torch.from_numpy(wl.H1[0]).to(gpu)
    chi, _, _, info = dm.susceptibility(H, A, wl.nocc, want_density=False, **_kw(prec))
    r_chi = float(dm.response(chi, H1)[0, 0])
    ec = cf.rel_frobenius(chi.double().cpu().numpy(), chiref)
    del chi
    d1, _, _, info1 = dm.susceptibility(H, H1, wl.nocc, spin=1.0, want_density=False, **_kw(prec))
    r_d1 = 2.0 * float(dm.response(d1, A)[0, 0])
    ed1 = cf.rel_frobenius(d1.double().cpu().numpy(), d1ref)
    print(f"\nwater N=7224 {prec}: M={info['m']} (D1 route M={info1['m']}) errchi={ec:.2e} errD1={ed1:.2e} "
          f"Tr[chi H1]={r_chi:.6f} ({abs(r_chi - rref) / abs(rref):.1e} of the value) "
          f"2Tr[A D1]={r_d1:.6f} ({abs(r_d1 - rref) / abs(rref):.1e})")
    # targets: 1e-5 for the FP32 path and refined runs, 1e-4 for
    # split products (the FP16 split measures 1.0e-5 here)
    tol = TOL_WATER[prec]
    assert ec <= tol and ed1 <= tol
    assert abs(r_chi - rref) <= tol * scale and abs(r_d1 - rref) <= tol * scale


def test_water_largest_accurate_projections(gpu, water301):
    """project = 2 on the largest shape: with Y projected in three terms and
    the correction's delta in two, the density-matrix route's dipole-weighted
    trace 2 Tr[A D1] meets the closed form to 1e-5 of the value, as the chi
    route does (with the cheaper projections it misses by 3.4e-5, measured)."""
    import torch

    import paper_2409_17033_amd as dm
    wl, chiref, d1ref, rref, scale = water301
    H = torch.from_numpy(wl.H).to(gpu)
    A = torch.from_numpy(wl.A[0]).to(gpu)
    H1 = torch.from_numpy(wl.H1[0]).to(gpu)
    kw = dict(_kw(HEADLINE), project=2)
    chi, _, _, info = dm.susceptibility(H, A, wl.nocc, want_density=False, **kw)
    r_chi = float(dm.response(chi, H1)[0, 0])
    ec = cf.rel_frobenius(chi.double().cpu().numpy(), chiref)
    del chi
    d1, _, _, _ = dm.susceptibility(H, H1, wl.nocc, spin=1.0, want_density=False, **kw)
    r_d1 = 2.0 * float(dm.response(d1, A)[0, 0])
    ed1 = cf.rel_frobenius(d1.double().cpu().numpy(), d1ref)
    print(f"\nwater N=7224 project=2: errchi={ec:.2e} errD1={ed1:.2e} "
          f"Tr[chi H1] {abs(r_chi - rref) / abs(rref):.1e}, 2Tr[A D1] {abs(r_d1 - rref) / abs(rref):.1e} of the value")
    assert ec <= 1e-5 and ed1 <= 1e-5
    assert abs(r_chi - rref) <= 1e-5 * abs(rref) and abs(r_d1 - rref) <= 1e-5 * abs(rref)
