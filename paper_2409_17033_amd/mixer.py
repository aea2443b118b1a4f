"""The learned mixer of the self-consistent response loop (Eq. CP_SCF).

A two-layer network of hidden width h with BF16 weights, applied site by site
(site i sees the residual and the on-site energies in a window of 2w + 1
sites, and its U_i), stands
in as the preconditioner of the loop: from the state v and residual r it
proposes v + mix r + (||r|| / sqrt(n)) net(sqrt(n) r / ||r||).  It is trained
on pairs the method itself produces: linear-mixing runs record (v_k, r_k);
with their converged state v* the target of x = sqrt(n) r_k / ||r_k|| is
t = sqrt(n) (v* - v_k - mix r_k) / ||r_k||, the exact correction to the
linear step.  Forward, loss gradient and Adam run in the library's kernels
(dmpt_mixer_*); this module owns the buffers.
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import check, load


class Mixer:
    def __init__(self, U, E, window: int = 32, hidden: int = 256, seed: int = 0):
        """U: (n,) float32 device tensor of on-site interactions, E: (n,) the
        on-site energies (diagonal of H0); both are per-site inputs."""
        lib = load()
        self.U = U.contiguous().float()
        self.E = E.contiguous().float()
        self.n, self.window, self.hidden = U.shape[0], window, hidden
        device = U.device
        count = int(lib.dmpt_mixer_param_count(window, hidden))
        if count == 0:
            check(1)
        self.count = count
        self.master = torch.empty(count, dtype=torch.float32, device=device)
        self.params = torch.empty(count, dtype=torch.int16, device=device)   # BF16 bit patterns
        self.adam_m = torch.zeros(count, dtype=torch.float32, device=device)
        self.adam_v = torch.zeros(count, dtype=torch.float32, device=device)
        self.steps = 0
        check(lib.dmpt_mixer_init(C.c_void_p(self.master.data_ptr()), C.c_void_p(self.params.data_ptr()),
                                  window, hidden, seed, C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def _ws(self, batch):
        nbytes = int(load().dmpt_mixer_workspace_bytes(self.n, self.window, self.hidden, batch))
        if nbytes == 0:
            check(1)
        return torch.empty(nbytes, dtype=torch.uint8, device=self.master.device)

    def params_float(self) -> torch.Tensor:
        """The BF16 parameters widened to FP32 (exact)."""
        return (self.params.to(torch.int32) << 16).view(torch.float32)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        x = x.contiguous().float()
        b = x.shape[0]
        y = torch.empty_like(x)
        ws = self._ws(b)
        check(load().dmpt_mixer_forward(C.c_void_p(self.params.data_ptr()), self.window, self.hidden,
                                        C.c_void_p(self.U.data_ptr()), C.c_void_p(self.E.data_ptr()), self.n,
                                        C.c_void_p(x.data_ptr()), b, C.c_void_p(y.data_ptr()),
                                        C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                        C.c_void_p(ws.data_ptr()), ws.numel()))
        return y

    def loss_grad(self, x: torch.Tensor, t: torch.Tensor):
        x, t = x.contiguous().float(), t.contiguous().float()
        b = x.shape[0]
        grad = torch.empty(self.count, dtype=torch.float32, device=x.device)
        loss = C.c_double()
        ws = self._ws(b)
        check(load().dmpt_mixer_loss_grad(C.c_void_p(self.params.data_ptr()), self.window, self.hidden,
                                          C.c_void_p(self.U.data_ptr()), C.c_void_p(self.E.data_ptr()), self.n,
                                          C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), b,
                                          C.c_void_p(grad.data_ptr()), C.byref(loss),
                                          C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                          C.c_void_p(ws.data_ptr()), ws.numel()))
        return loss.value, grad

    def train(self, x: torch.Tensor, t: torch.Tensor, steps: int, batch: int = 64, lr: float = 1e-3):
        """Adam steps over minibatches of consecutive pairs; returns the loss per step.
        The step counter continues across calls only through the moment buffers
        (each call restarts the bias correction at 1)."""
        x, t = x.contiguous().float(), t.contiguous().float()
        npairs = x.shape[0]
        hist = (C.c_double * steps)()
        ws = self._ws(batch)
        check(load().dmpt_mixer_train(C.c_void_p(self.master.data_ptr()), C.c_void_p(self.params.data_ptr()),
                                      C.c_void_p(self.adam_m.data_ptr()), C.c_void_p(self.adam_v.data_ptr()),
                                      self.window, self.hidden, C.c_void_p(self.U.data_ptr()),
                                      C.c_void_p(self.E.data_ptr()), self.n,
                                      C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                      npairs, batch, steps, lr, hist,
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                      C.c_void_p(ws.data_ptr()), ws.numel()))
        self.steps += steps
        return list(hist)


def _rows_ws(rows: int, device):
    nbytes = int(load().dmpt_mixer_rows_workspace_bytes(rows))
    if nbytes == 0:
        check(1)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _pairs(v, r, residual, vstar, mix: float, min_residual: float, drop_last: bool):
    """(x, t) of the recorded states whose relative residual is at least
    min_residual (dmpt_mixer_pairs): x = sqrt(n) r / ||r||,
    t = sqrt(n) (v* - v - mix r) / ||r||."""
    v, r, vstar = v.contiguous().float(), r.contiguous().float(), vstar.contiguous().float()
    k, n = v.shape
    res = (C.c_double * k)(*[float(x) for x in residual[:k]])
    x = torch.empty((k, n), dtype=torch.float32, device=v.device)
    t = torch.empty((k, n), dtype=torch.float32, device=v.device)
    count = C.c_int32(0)
    ws = _rows_ws(k, v.device)
    check(load().dmpt_mixer_pairs(C.c_void_p(v.data_ptr()), C.c_void_p(r.data_ptr()), res, k, n,
                                  C.c_void_p(vstar.data_ptr()), mix, min_residual, 1 if drop_last else 0,
                                  C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), k, C.byref(count),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                  C.c_void_p(ws.data_ptr()), ws.numel()))
    return x[:count.value], t[:count.value]


def _shuffle(x, t, seed: int):
    """The rows of (x, t) in one random order (dmpt_mixer_shuffle)."""
    x, t = x.contiguous(), t.contiguous()
    npairs, n = x.shape
    xo, to = torch.empty_like(x), torch.empty_like(t)
    ws = _rows_ws(npairs, x.device)
    check(load().dmpt_mixer_shuffle(C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), npairs, n, seed,
                                    C.c_void_p(xo.data_ptr()), C.c_void_p(to.data_ptr()),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                    C.c_void_p(ws.data_ptr()), ws.numel()))
    return xo, to


def training_pairs(H0, U, observables, nocc: int, *, mix: float = 0.3, tol: float = 1e-6, max_iter: int = 400,
                   min_residual: float = 1e-5, return_fixed_points: bool = False, **kw):
    """Pairs (x, t) from linear-mixing runs of dmpt_scf_response, one run per
    observable: x_k = sqrt(n) r_k / ||r_k||, t_k = sqrt(n) (v* - v_k - mix r_k) / ||r_k||,
    v* the run's last state.  States whose relative residual is below
    min_residual are left out: their targets are dominated by the rounding
    noise of v* (the FP32 loop's residual floor is ~1e-7)."""
    from . import scf_response
    xs, ts, vstars = [], [], []
    for a in observables:
        _, sinfo, _, v, r = scf_response(H0, U, a, nocc, mixer="linear", mix=mix, tol=tol, max_iter=max_iter,
                                         record=True, **kw)
        vstar = v[-1:].clone()
        x, t = _pairs(v, r, sinfo["residual"], vstar, mix, min_residual, drop_last=True)
        xs.append(x)
        ts.append(t)
        vstars.append(vstar)
    out = (torch.cat(xs), torch.cat(ts))
    return out + (vstars,) if return_fixed_points else out


def train_mixer(H0, U, observables, nocc: int, *, window: int = 32, hidden: int = 256, passes: int = 2,
                steps: int = 6000, batch: int = 64, lr: float = 1e-3, mix: float = 0.3, tol: float = 1e-6,
                max_iter: int = 400, collect_iter: int = 100, min_residual: float = 1e-5, seed: int = 11, **kw):
    """Train a mixer for the loop of (H0, U) on the method's own pairs.

    Pass 0 trains on the states of linear-mixing runs (training_pairs).  A
    network trained only there meets, once it is used, residuals that its own
    earlier steps left behind, which linear mixing never produces; so each
    further pass runs the learned loop on the training observables, labels
    every state it visits with the exact correction toward that observable's
    fixed point v* (from the linear run), adds those pairs to the set and
    trains a fresh network on the union (data aggregation; Ross, Gordon &
    Bagnell, 2011).  Every network is scored by its mean number of loop
    evaluations over the training observables and the best one is returned,
    with a report {passes: [(pairs, loss, mean evaluations)], chosen: index}.
    The learned runs stop after collect_iter evaluations (a poor early network
    would otherwise spend max_iter on each observable).
    """
    from . import scf_response
    x, t, vstars = training_pairs(H0, U, observables, nocc, mix=mix, tol=tol, max_iter=max_iter,
                                  min_residual=min_residual, return_fixed_points=True, **kw)
    report, best = {"passes": []}, None
    E = H0.diagonal().contiguous().float()      # on-site energies (a network input)
    for rnd in range(passes + 1):
        net = Mixer(U, E, window=window, hidden=hidden, seed=seed + rnd)
        hist = net.train(x, t, steps=steps, batch=batch, lr=lr)
        loss = sum(hist[-100:]) / len(hist[-100:])
        xs, ts, evals = [x], [t], []
        for a, vstar in zip(observables, vstars):
            _, sinfo, _, v, r = scf_response(H0, U, a, nocc, mixer="learned", net=net, mix=mix, tol=tol,
                                             max_iter=collect_iter, record=True, raise_on_error=False, **kw)
            evals.append(sinfo["iters"])
            if rnd < passes:
                xn, tn = _pairs(v, r, sinfo["residual"], vstar, mix, min_residual, drop_last=False)
                xs.append(xn)
                ts.append(tn)
        score = sum(evals) / len(evals)
        report["passes"].append((int(x.shape[0]), loss, score))
        if best is None or score < best[1]:
            best = (net, score, rnd)
        if rnd < passes:
            x, t = _shuffle(torch.cat(xs), torch.cat(ts), seed * 1000003 + rnd)
    report["chosen"] = best[2]
    return best[0], report
