"""Differentiation path (the backward sweep behind torch.autograd), config 3:
N = 2048 banded gapped H (config-2 recipe at N = 2048), FP32, checkpoint
interval 8, 16 random symmetric Frobenius-normalised observables, 32 random
H1, central finite differences with h = 1e-3.

References: the FP64 Daleckii-Krein closed form (oracle) for chi, and finite
differences of the GPU forward pass itself.  FD in FP32 is noise-limited
(D carries ~1e-6 relative error), so the FD check is stated against the
Cauchy-Schwarz scale ||chi_k||_F ||H1||_F of each response.
"""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf

pytestmark = pytest.mark.gpu

N, K, P, H_STEP, CKPT = 2048, 16, 32, 1e-3, 8


@pytest.fixture(scope="module")
def c3():
    wl = W.banded_gapped(N, cfg=3, nobs=K, observable="random", npert=P, cache=False)
    chis = cf.first_order_responses(wl.H.astype(np.float64), wl.A.astype(np.float64), wl.nocc)
    return wl, chis                   # spin-less chi' per observable


def test_autograd_matches_closed_form(gpu, c3):
    import torch

    from paper_2409_17033_amd.autograd import density
    wl = c3[0]
    H = torch.from_numpy(wl.H).to(gpu).requires_grad_(True)
    A = torch.from_numpy(wl.A[0]).to(gpu)
    D = density(H, wl.nocc, ckpt_interval=CKPT)
    loss = (A * D).sum()              # Tr[A D] for symmetric A
    loss.backward()
    g = H.grad.double().cpu().numpy()
    ref = c3[1][0]
    err = cf.rel_frobenius(g, ref)
    print(f"\nautograd chi err {err:.2e}")
    assert err <= 1e-5


def test_checkpointed_adjoint_is_bitwise_unchanged(gpu, c3):
    """Recomputing X_n between checkpoints reproduces them exactly, so the
    swept chi does not depend on the checkpoint interval."""
    import torch

    import paper_2409_17033_amd as dm
    wl = c3[0]
    H = torch.from_numpy(wl.H).to(gpu)
    A = torch.from_numpy(wl.A[:2]).to(gpu)
    out = {}
    for k in (0, 1, CKPT, 5):
        chi, _, _, info = dm.susceptibility(H, A, wl.nocc, sweep="adjoint", ckpt_interval=k)
        out[k] = chi.cpu().numpy()
    for k in (1, CKPT, 5):
        np.testing.assert_array_equal(out[k], out[0])


def test_batched_backward_16_observables(gpu, c3):
    import torch

    from paper_2409_17033_amd.autograd import observable_gradients
    wl = c3[0]
    H = torch.from_numpy(wl.H).to(gpu)
    A = torch.from_numpy(wl.A).to(gpu)
    chi, D, a0, info = observable_gradients(H, A, wl.nocc, ckpt_interval=CKPT)
    c = chi.double().cpu().numpy()
    errs = [cf.rel_frobenius(c[k], 2.0 * c3[1][k]) for k in range(K)]
    print(f"\nbatched adjoint M={info['m']} max chi err {max(errs):.2e}")
    assert max(errs) <= 1e-5


def test_finite_differences(gpu, c3):
    import torch

    import paper_2409_17033_amd as dm
    wl = c3[0]
    H = torch.from_numpy(wl.H).to(gpu)
    A = torch.from_numpy(wl.A).to(gpu)
    chi, _, _, _ = dm.susceptibility(H, A, wl.nocc, sweep="adjoint", ckpt_interval=CKPT, spin=1.0)
    resp = dm.response(chi, torch.from_numpy(wl.H1).to(gpu))          # [K, P]
    Ad = A.double()
    worst = 0.0
    for p in range(P):
        h1 = torch.from_numpy(wl.H1[p]).to(gpu)
        Dp, _ = dm.sp2_density((H + H_STEP * h1).contiguous(), wl.nocc)
        Dm, _ = dm.sp2_density((H - H_STEP * h1).contiguous(), wl.nocc)
        fd = ((Ad * (Dp.double() - Dm.double())).sum(dim=(1, 2)) / (2 * H_STEP)).cpu().numpy()
        scale = torch.linalg.norm(chi.double(), dim=(1, 2)).cpu().numpy() * float(torch.linalg.norm(h1))
        worst = max(worst, float(np.max(np.abs(fd - resp[:, p]) / scale)))
    print(f"\nFD worst |fd - Tr[chi H1]| / (||chi|| ||H1||) = {worst:.2e}")
    assert worst <= 2e-3
