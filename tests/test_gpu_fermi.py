"""Finite electronic temperature (Sec. V.B) on the GPU through the C ABI,
against the FP64 oracle (oracle/fermi.py: Fermi function with the canonical
chemical potential, Daleckii-Krein susceptibility with the mu_1 shift).

Cases: config-5-like gapless banded H (half-bandwidth 256 scaled down to
n = 1000, 4 observables batched) at kT = 0.01 and 0.05, canonical and grand
canonical; the low-temperature limit on a gapped H equals the zero-temperature
path; the duality Tr[chi_A B] = Tr[A chi_B]; batched observables equal single
runs bit for bit; FP32 and FP16 double-half split products.  Tolerance
2e-5 relative Frobenius: FP32 (or 22-bit split) products through
m ~ 16 doubling steps, each with up to five Newton-Schulz products, plus the
linearised start (relative (beta w / 2^m)^2 / 12 <= 2e-6 with the default m).
"""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf
from oracle import fermi as fo

pytestmark = pytest.mark.gpu

TOL = 2e-5


def _dev(x, gpu):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(gpu)


@pytest.fixture(scope="module")
def c5():
    return W.banded_gapless(1000, half_bandwidth=256, nobs=4)


@pytest.mark.parametrize("prec", ["fp32", "split_fp16"])
@pytest.mark.parametrize("kt", [0.01, 0.05])
def test_canonical_matches_oracle(gpu, c5, kt, prec):
    import paper_2409_17033_amd as dm
    wl = c5
    h = wl.H.astype(np.float64)
    chi, D, a0, info = dm.susceptibility_fermi(_dev(wl.H, gpu), _dev(wl.A, gpu), wl.nocc, kt, bounds="gershgorin",
                                               precision=prec)
    d_ref, mu_ref = fo.fermi_density(h, wl.nocc, 1.0 / kt)
    assert abs(info["mu"] - mu_ref) <= 1e-4 * (info["emax"] - info["emin"])
    ed = cf.rel_frobenius(D.double().cpu().numpy(), d_ref)
    errs = []
    for k in range(wl.A.shape[0]):
        ref, _, mu1 = fo.fermi_susceptibility(h, wl.A[k].astype(np.float64), wl.nocc, 1.0 / kt, spin=2.0)
        errs.append(cf.rel_frobenius(chi[k].double().cpu().numpy(), ref))
        assert abs(info["mu1"][k] - mu1) <= 1e-4 * max(1.0, abs(mu1))
        assert abs(a0[k] - 2.0 * np.sum(wl.A[k].astype(np.float64) * d_ref)) <= TOL * np.linalg.norm(d_ref) * 2
        assert abs(float(chi[k].double().trace())) <= 1e-4 * np.linalg.norm(ref)
    print(f"\n{prec} kT={kt}: m={info['doublings']} newton={info['newton']} products={info['products']} mu={info['mu']:.6f} "
          f"errD {ed:.2e} errchi {max(errs):.2e} {info['elapsed_ms']:.1f} ms")
    assert ed <= TOL and max(errs) <= TOL
    assert abs(info["trace_d"] - wl.nocc) <= 1e-6 * wl.n + 1e-9


def test_grand_canonical_matches_oracle(gpu, c5):
    import paper_2409_17033_amd as dm
    wl = c5
    h = wl.H.astype(np.float64)
    kt, mu = 0.02, 0.1
    chi, D, _, info = dm.susceptibility_fermi(_dev(wl.H, gpu), _dev(wl.A[0], gpu), wl.nocc, kt, canonical=False,
                                              mu=mu, bounds="gershgorin")
    w, v = np.linalg.eigh(h)
    d_ref = (v * fo.occupations(w, mu, 1.0 / kt)) @ v.T
    lw = fo.loewner_fermi(w, mu, 1.0 / kt)
    ref = 2.0 * v @ (lw * (v.T @ wl.A[0].astype(np.float64) @ v)) @ v.T
    assert info["mu"] == mu and info["newton"] == 0
    assert cf.rel_frobenius(D.double().cpu().numpy(), d_ref) <= TOL
    assert cf.rel_frobenius(chi.double().cpu().numpy(), ref) <= TOL


def test_low_temperature_limit_is_zero_temperature(gpu):
    import paper_2409_17033_amd as dm
    wl = W.dense_gapped(300, nocc=117, cfg=11)     # gap 0.2
    h = wl.H.astype(np.float64)
    chi, D, _, info = dm.susceptibility_fermi(_dev(wl.H, gpu), _dev(wl.A[0], gpu), wl.nocc, 0.002)
    assert cf.rel_frobenius(D.double().cpu().numpy(), cf.density_matrix(h, wl.nocc)) <= TOL
    ref0 = cf.susceptibility(h, wl.A[0].astype(np.float64), wl.nocc, spin=2.0)
    assert cf.rel_frobenius(chi.double().cpu().numpy(), ref0) <= TOL


def test_duality_and_batching(gpu, c5):
    """Tr[chi_A B] = Tr[A chi_B] (the canonical susceptibility is self-adjoint),
    and a batch of observables reproduces single runs bit for bit."""
    import torch

    import paper_2409_17033_amd as dm
    wl = c5
    H, A = _dev(wl.H, gpu), _dev(wl.A, gpu)
    chi, _, _, _ = dm.susceptibility_fermi(H, A, wl.nocc, 0.01, bounds="gershgorin")
    lhs = float((chi[0].double() * A[1].double()).sum())
    rhs = float((A[0].double() * chi[1].double()).sum())
    assert abs(lhs - rhs) <= 1e-4 * max(abs(lhs), 1e-3 * float(chi[0].double().norm()))
    one, _, _, _ = dm.susceptibility_fermi(H, A[2].contiguous(), wl.nocc, 0.01, bounds="gershgorin")
    assert torch.equal(one, chi[2])


@pytest.fixture(scope="module")
def c5_full():
    """Config 5 at its size: N = 16384, gapless banded H (half-bandwidth 256),
    kT = 0.01; four of its observables (the batch shape is what matters; the
    32 of the full configuration are timed by bench.py --extra fermi)."""
    return W.banded_gapless(16384, half_bandwidth=256, nobs=4)


def test_config5_full_size(gpu, c5_full):
    """N = 16384 with the three-term BF16 split (config 5's split-BF16
    products) and FP32, four observables in one batch: the electron count,
    Tr chi = 0 (the mu_1 shift), the self-adjointness Tr[chi_A B] = Tr[A chi_B]
    of the canonical susceptibility, and the two precisions agreeing on D, mu
    and chi.  No closed form at this size (an FP64 eigendecomposition of
    16384 x 16384 takes minutes): the same checks pass against the oracle at
    n = 1000 above."""
    import torch

    import paper_2409_17033_amd as dm
    wl = c5_full
    H, A = _dev(wl.H, gpu), _dev(wl.A, gpu)
    out = {}
    for prec in ("split3_bf16", "fp32"):
        chi, D, a0, info = dm.susceptibility_fermi(H, A, wl.nocc, 0.01, precision=prec)
        torch.cuda.synchronize()
        cd = chi.double()
        tr = max(abs(float(cd[k].trace())) / float(cd[k].norm()) for k in range(4))
        lhs = float((cd[0] * A[1].double()).sum())
        rhs = float((A[0].double() * cd[1]).sum())
        dual = abs(lhs - rhs) / max(abs(lhs), 1e-3 * float(cd[0].norm()))
        print(f"\nN=16384 {prec}: m={info['doublings']} newton={info['newton']} products={info['products']} "
              f"mu={info['mu']:.6f} TrD-N={info['trace_d'] - wl.nocc:.2e} Tr chi {tr:.1e} duality {dual:.1e} "
              f"{info['elapsed_ms'] / 1e3:.1f} s", flush=True)
        assert abs(info["trace_d"] - wl.nocc) <= 1e-6 * wl.n
        assert tr <= 1e-5 and dual <= 1e-4
        out[prec] = (chi.cpu(), D.cpu(), info["mu"])
        del chi, D, cd
        torch.cuda.empty_cache()
    (c3, d3, mu3), (c32, d32, mu32) = out["split3_bf16"], out["fp32"]
    ec = float((c3.double() - c32.double()).norm() / c32.double().norm())
    ed = float((d3.double() - d32.double()).norm() / d32.double().norm())
    print(f"split3_bf16 vs fp32: chi {ec:.1e} D {ed:.1e} mu {abs(mu3 - mu32):.1e}")
    assert ec <= 1e-4 and ed <= 1e-5 and abs(mu3 - mu32) <= 1e-6
