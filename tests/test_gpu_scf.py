"""Self-consistent response (Eq. CP_SCF) and its learned mixer on the GPU
(config 4: N = 1024 banded gapped H0, U_i ~ U(0.5, 1.5), external field
H1 = diag(N(0, 0.01^2)), FP32, residual target 1e-6; the FP32 loop's
residual floor is ~1.5e-7).

References: the FP64 oracle (oracle/scf.py, oracle/mlp.py) for the loop's
result (at N = 256 and at config 4's N = 1024, every mixer) and for the
network's forward pass, gradient and Adam step; the
GPU's own duality Tr[chi_A H1] = Tr[A chi_H1] (both self-consistent).
"""
import numpy as np
import pytest

import workloads as W
from oracle import closed_form as cf
from oracle import mlp as omlp
from oracle import scf as oscf

pytestmark = pytest.mark.gpu


def _bf16(t):
    """BF16 parameter tensor (int16 bit patterns) -> float64 numpy values."""
    return (t.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _u(n, seed):
    import torch
    g = torch.Generator().manual_seed(seed)
    return 0.5 + torch.rand(n, generator=g)


def _e(n, seed):
    import torch
    g = torch.Generator().manual_seed(seed + 100)
    return 2.0 * torch.rand(n, generator=g) - 1.0


@pytest.mark.parametrize("n,w,h,b", [(256, 8, 64, 16), (1024, 32, 256, 8), (37, 40, 16, 3)])
def test_mixer_forward_and_gradient(gpu, n, w, h, b):
    """Site-local network on (B, n) states: forward, loss and gradient
    against the FP64 oracle with the same BF16 parameters (the last case has
    a window wider than the system and a ragged site count)."""
    import torch

    from paper_2409_17033_amd.mixer import Mixer
    u, en = _u(n, 9), _e(n, 9)
    net = Mixer(u.to(gpu), en.to(gpu), window=w, hidden=h, seed=3)
    g = torch.Generator().manual_seed(1)
    x = torch.randn(b, n, generator=g).to(gpu)
    t = torch.randn(b, n, generator=g).to(gpu)
    p = _bf16(net.params)
    un, enn = u.double().numpy(), en.double().numpy()
    y = net.forward(x).double().cpu().numpy()
    yref, _, _ = omlp.forward(p, x.double().cpu().numpy(), un, enn, w, h)
    assert cf.rel_frobenius(y, yref) <= 1e-5
    loss, grad = net.loss_grad(x, t)
    lref, gref = omlp.loss_grad(p, x.double().cpu().numpy(), t.double().cpu().numpy(), un, enn, w, h)
    assert abs(loss - lref) <= 1e-5 * lref
    assert cf.rel_frobenius(grad.double().cpu().numpy(), gref) <= 1e-4


def test_mixer_pairs_and_shuffle(gpu):
    """Training pairs labelled by dmpt_mixer_pairs against the definition
    x = sqrt(n) r / ||r||, t = sqrt(n) (v* - v - mix r) / ||r|| computed in
    FP64 here from the same FP32 records; rows below min_residual and, with
    drop_last, the last row are left out.  dmpt_mixer_shuffle returns the
    same (x, t) pairs in one seeded order."""
    import torch

    from paper_2409_17033_amd.mixer import _pairs, _shuffle
    rng = np.random.default_rng(5)
    k, n, mix = 7, 301, 0.3
    v = rng.normal(size=(k, n)).astype(np.float32)
    r = (rng.normal(size=(k, n)) * 10.0 ** -np.arange(k)[:, None]).astype(np.float32)
    vstar = rng.normal(size=(1, n)).astype(np.float32)
    residual = [10.0 ** -j for j in range(k)]
    for drop_last in (False, True):
        x, t = _pairs(torch.from_numpy(v).to(gpu), torch.from_numpy(r).to(gpu), residual,
                      torch.from_numpy(vstar).to(gpu), mix, 1e-5, drop_last)
        keep = [j for j in range(k) if residual[j] >= 1e-5 and not (drop_last and j == k - 1)]
        v64, r64, s64 = v.astype(np.float64), r.astype(np.float64), vstar.astype(np.float64)[0]
        rn = np.linalg.norm(r64[keep], axis=1, keepdims=True) / np.sqrt(n)
        xref = r64[keep] / rn
        tref = (s64 - v64[keep] - mix * r64[keep]) / rn
        assert x.shape == (len(keep), n)
        assert cf.rel_frobenius(x.double().cpu().numpy(), xref) <= 1e-6
        assert cf.rel_frobenius(t.double().cpu().numpy(), tref) <= 1e-6
    xs, ts = _shuffle(x, t, 11)
    xs2, ts2 = _shuffle(x, t, 11)
    assert torch.equal(xs, xs2) and torch.equal(ts, ts2)
    xa, ta, xb, tb = (q.cpu().numpy() for q in (x, t, xs, ts))
    order = [next(i for i in range(len(xa)) if np.array_equal(xa[i], row)) for row in xb]
    assert sorted(order) == list(range(len(xa)))             # a permutation of the rows
    assert all(np.array_equal(ta[i], tb[j]) for j, i in enumerate(order))   # pairs kept together


def test_mixer_adam_step(gpu):
    import torch

    from paper_2409_17033_amd.mixer import Mixer
    n, w, h, b = 128, 4, 32, 8
    u, en = _u(n, 4), _e(n, 4)
    net = Mixer(u.to(gpu), en.to(gpu), window=w, hidden=h, seed=5)
    g = torch.Generator().manual_seed(2)
    x = torch.randn(b, n, generator=g).to(gpu)
    t = torch.randn(b, n, generator=g).to(gpu)
    p0 = net.master.double().cpu().numpy()
    _, gref = omlp.loss_grad(_bf16(net.params), x.double().cpu().numpy(), t.double().cpu().numpy(),
                             u.double().numpy(), en.double().numpy(), w, h)
    net.train(x, t, steps=1, batch=b, lr=1e-3)
    p1 = net.master.double().cpu().numpy()
    pref, _, _ = omlp.adam_step(p0, gref, np.zeros_like(p0), np.zeros_like(p0), 1, lr=1e-3)
    big = np.abs(gref) > 1e-5                     # where the sign of the step is not in doubt
    np.testing.assert_allclose((p1 - p0)[big], (pref - p0)[big], rtol=1e-3, atol=1e-7)
    # the BF16 copy is the rounded master
    np.testing.assert_allclose(_bf16(net.params), p1, rtol=2 ** -8)


def test_training_reduces_loss(gpu):
    import torch

    from paper_2409_17033_amd.mixer import Mixer
    n, w, h = 64, 3, 32
    net = Mixer(_u(n, 6).to(gpu), _e(n, 6).to(gpu), window=w, hidden=h, seed=7)
    g = torch.Generator().manual_seed(3)
    x = torch.randn(256, n, generator=g)
    kern = torch.tensor([0.1, -0.3, 0.5, 1.0, 0.5, -0.3, 0.1])
    t = torch.nn.functional.conv1d(x[:, None, :], kern[None, None, :], padding=3)[:, 0]
    hist = net.train(x.to(gpu), t.contiguous().to(gpu), steps=400, batch=32, lr=3e-3)
    assert hist[-1] < 0.25 * hist[0]


def _scf_small():
    wl, u, _ = W.scf_system(256, cfg=14, ntrain=0)
    return wl, u


def test_scf_matches_oracle(gpu):
    import torch

    import paper_2409_17033_amd as dm
    wl, u = _scf_small()
    h0, a = wl.H.astype(np.float64), wl.A[0].astype(np.float64)
    ref, _, _ = oscf.scf_susceptibility(h0, a, u.astype(np.float64), wl.nocc, spin=2.0, tol=1e-12)
    for mixer in ("linear", "anderson"):
        chi, sinfo, _ = dm.scf_response(torch.from_numpy(wl.H).to(gpu), torch.from_numpy(u).to(gpu),
                                        torch.from_numpy(wl.A[0]).to(gpu), wl.nocc, mixer=mixer, tol=1e-6)
        err = cf.rel_frobenius(chi.double().cpu().numpy(), ref)
        print(f"\nscf {mixer}: evaluations {sinfo['iters']} err {err:.2e}")
        assert sinfo["converged"] and err <= 1e-5


def test_scf_no_interaction_is_plain_susceptibility(gpu):
    import torch

    import paper_2409_17033_amd as dm
    wl, u = _scf_small()
    H, A = torch.from_numpy(wl.H).to(gpu), torch.from_numpy(wl.A[0]).to(gpu)
    chi, sinfo, _ = dm.scf_response(H, torch.zeros_like(torch.from_numpy(u)).to(gpu), A, wl.nocc, mix=1.0)
    chi0, _, _, _ = dm.susceptibility(H, A, wl.nocc, sweep="adjoint")
    assert sinfo["iters"] <= 2
    np.testing.assert_array_equal(chi.cpu().numpy(), chi0.cpu().numpy())


@pytest.fixture(scope="module")
def c4():
    return W.scf_system(1024, cfg=4, ntrain=80)


@pytest.fixture(scope="module")
def c4_oracle(c4):
    """The FP64 oracle's self-consistent chi of config 4's A (the paper's
    linear loop on full matrices, Eq. CP_SCF, stopped when the update falls
    below 1e-11 of ||L[A]||_F; about 70 iterations)."""
    wl, u, _ = c4
    h0, a = wl.H.astype(np.float64), wl.A[0].astype(np.float64)
    scale = np.linalg.norm(oscf.FirstOrder(h0, wl.nocc)(a))
    ref, it, _ = oscf.scf_susceptibility(h0, a, u.astype(np.float64), wl.nocc, spin=2.0, tol=1e-11 * scale)
    return ref


@pytest.mark.parametrize("mixer", ["linear", "anderson"])
def test_scf_config4_matches_oracle(gpu, c4, c4_oracle, mixer):
    """Config 4 at its size (N = 1024): the self-consistent chi of the GPU
    loop against the oracle's fixed point."""
    import torch

    import paper_2409_17033_amd as dm
    wl, u, _ = c4
    chi, sinfo, _ = dm.scf_response(torch.from_numpy(wl.H).to(gpu), torch.from_numpy(u).to(gpu),
                                    torch.from_numpy(wl.A[0]).to(gpu), wl.nocc, mixer=mixer, tol=1e-6)
    err = cf.rel_frobenius(chi.double().cpu().numpy(), c4_oracle)
    print(f"\nconfig 4 scf {mixer}: evaluations {sinfo['iters']} err {err:.2e}")
    assert sinfo["converged"] and err <= 1e-5


def test_scf_duality_config4(gpu, c4):
    """Tr[chi_A H1] = Tr[A chi_H1]: the self-consistent susceptibility of A and
    the self-consistent density response to H1 (the same loop with A := H1)."""
    import torch

    import paper_2409_17033_amd as dm
    wl, u, _ = c4
    H, U = torch.from_numpy(wl.H).to(gpu), torch.from_numpy(u).to(gpu)
    A, H1 = torch.from_numpy(wl.A[0]).to(gpu), torch.from_numpy(wl.H1[0]).to(gpu)
    chi_a, s1, _ = dm.scf_response(H, U, A, wl.nocc, tol=1e-6)
    chi_h, s2, _ = dm.scf_response(H, U, H1, wl.nocc, tol=1e-6)
    lhs = float((chi_a.double() * H1.double()).sum())
    rhs = float((A.double() * chi_h.double()).sum())
    print(f"\nduality {lhs:.8e} {rhs:.8e} evals {s1['iters']} {s2['iters']}")
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)


@pytest.mark.timeout(600)
def test_learned_mixer_gain_config4(gpu, c4, c4_oracle):
    """Train the mixer on the method's own pairs from 72 training observables
    (linear-mixing states, then two passes of states the learned loop visits;
    over 2000 pairs), then solve for held-out observables (A and 8 more) with
    linear, Anderson and learned mixing to residual 1e-6: the learned loop
    must reach the same chi as linear mixing in fewer evaluations."""
    import torch

    import paper_2409_17033_amd as dm
    from paper_2409_17033_amd.mixer import train_mixer
    wl, u, train = c4
    H, U = torch.from_numpy(wl.H).to(gpu), torch.from_numpy(u).to(gpu)
    obs = [torch.from_numpy(a).to(gpu) for a in train]
    net, report = train_mixer(H, U, obs[:72], wl.nocc, window=32, hidden=256, passes=2)
    print(f"\ntraining passes (pairs, loss, mean evaluations): {report['passes']}, chosen {report['chosen']}")
    held = [torch.from_numpy(wl.A[0]).to(gpu)] + obs[72:80]
    ev = {"linear": [], "anderson": [], "learned": [], "learned_anderson": []}
    for j, a in enumerate(held):
        chis = {}
        for mixer in ev:
            chi, sinfo, _ = dm.scf_response(H, U, a, wl.nocc, mixer=mixer, net=net, tol=1e-6, max_iter=400)
            assert sinfo["converged"], (j, mixer)
            ev[mixer].append(sinfo["iters"])
            chis[mixer] = chi.double().cpu().numpy()
        for k in ("anderson", "learned", "learned_anderson"):
            assert cf.rel_frobenius(chis[k], chis["linear"]) <= 1e-5
        if j == 0:   # A: every mixer's chi against the oracle's fixed point
            errs = {k: cf.rel_frobenius(c, c4_oracle) for k, c in chis.items()}
            print(f"\nconfig 4 A, error against the oracle: {errs}")
            assert max(errs.values()) <= 1e-5
    print("evaluations to 1e-6 on held-out observables: " + "; ".join(f"{k} {v}" for k, v in ev.items()))
    assert report["passes"][-1][0] >= 2000
    assert sum(ev["learned"]) < 0.75 * sum(ev["linear"])
    # the network as Anderson's preconditioner beats Anderson itself
    assert sum(ev["learned_anderson"]) < 0.85 * sum(ev["anderson"])
