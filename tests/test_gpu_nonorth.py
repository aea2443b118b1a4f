"""Non-orthonormal basis (Sec. V.A) on the GPU through the C ABI, against
the FP64 oracle (oracle/nonorth.py, itself pinned to the generalised
eigenproblem): D = Z D_perp Z^T, chi_perp, chi_ao = Z chi_perp Z^T and a0,
for Loewdin and Cholesky inverse factors of an SPD overlap near I, on a
ragged size (n = 300) and a banded case (n = 1000); the identity factor
reproduces the orthonormal path bit for bit."""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf
from oracle import nonorth as no

pytestmark = pytest.mark.gpu


def _overlap(n, seed):
    rng = np.random.default_rng([17033, 40, n, seed])
    g = np.zeros((n, n))
    for d in range(1, 4):                          # short-range overlap between neighbours
        v = rng.uniform(0.0, 0.15, size=n - d)
        g += np.diag(v, d) + np.diag(v, -d)
    return np.eye(n) + g


def _dev(x, gpu):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(gpu)


@pytest.mark.parametrize("case", ["dense300", "band1000"])
@pytest.mark.parametrize("factor", ["loewdin", "cholesky"])
@pytest.mark.parametrize("prec", ["fp32", "split_fp16"])
def test_nonorth_matches_oracle(gpu, case, factor, prec):
    import paper_2409_17033_amd as dm
    wl = W.dense_gapped(300, nocc=117, cfg=11) if case == "dense300" else \
        W.banded_gapped(1000, nocc=500, cfg=12, cache=False)
    n = wl.n
    s = _overlap(n, 1)
    z = no.loewdin_factor(s) if factor == "loewdin" else no.cholesky_factor(s)
    z32 = z.astype(np.float32).astype(np.float64)
    h, a = wl.H.astype(np.float64), wl.A[0].astype(np.float64)
    d_ref, chip_ref, chiao_ref, a0_ref = no.nonorth_response(h, z32, a, wl.nocc, spin=2.0)
    chi_p, chi_ao, D, a0, info = dm.susceptibility_nonorth(_dev(wl.H, gpu), _dev(z32, gpu), _dev(wl.A[0], gpu),
                                                           wl.nocc, precision=prec)
    ed = cf.rel_frobenius(D.double().cpu().numpy(), d_ref)
    ep = cf.rel_frobenius(chi_p.double().cpu().numpy(), chip_ref)
    ea = cf.rel_frobenius(chi_ao.double().cpu().numpy(), chiao_ref)
    print(f"\n{case} {factor} {prec}: M={info['m']} errD {ed:.2e} chi_perp {ep:.2e} chi_ao {ea:.2e}")
    assert ed <= 1e-5 and ep <= 1e-5 and ea <= 1e-5
    assert abs(a0[0] - a0_ref) <= 1e-5 * np.linalg.norm(a) * np.linalg.norm(d_ref)
    # the density also solves the generalised eigenproblem of (H, S) (Z enters only through its rounding)
    assert cf.rel_frobenius(D.double().cpu().numpy(), no.generalized_density(h, s, wl.nocc)) <= 1e-4


def test_identity_factor_is_the_orthonormal_path(gpu):
    import torch

    import paper_2409_17033_amd as dm
    wl = W.dense_gapped(300, nocc=117, cfg=11)
    H, A = _dev(wl.H, gpu), _dev(wl.A[0], gpu)
    eye = torch.eye(wl.n, dtype=torch.float32, device=gpu)
    chi_p, chi_ao, D, a0, _ = dm.susceptibility_nonorth(H, eye, A, wl.nocc, precision="split_fp16")
    chi, D0, a00, _ = dm.susceptibility(H, A, wl.nocc, precision="split_fp16")
    assert torch.equal(chi_p, chi) and torch.equal(chi_ao, chi) and torch.equal(D, D0)
    assert a0[0] == a00[0]
