"""Differentiable SP2 density matrix: the backward sweep as a torch backward pass.

forward   D = theta(mu I - H) by the SP2 recursion (Eq. DM0, dmpt_sp2_density).
backward  For a loss L(D) with G = dL/dD, dL/dH is the susceptibility of the
          "observable" G, chi_G = dTr[G D]/dH (Eq. Suscept with spin 1),
          computed by dmpt_susceptibility with the backward sweep of Eq. DM2:
          the recursion is run again (it is deterministic, so it takes the
          same sigma sequence), keeping X_n every `ckpt_interval` steps; the
          sweep recomputes the steps between checkpoints from the recorded
          sigma_n before it uses them.  Only the symmetric part of G enters
          (D is symmetric), which the library forms itself.

Both passes run in the HIP library; this module only marshals arguments.
"""
from __future__ import annotations

import torch

from . import sp2_density, susceptibility


class SP2Density(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H, nocc, ckpt_interval, opts):
        D, _ = sp2_density(H, nocc, **opts)
        ctx.save_for_backward(H)
        ctx.nocc, ctx.ckpt, ctx.opts = nocc, ckpt_interval, opts
        return D

    @staticmethod
    def backward(ctx, gD):
        (H,) = ctx.saved_tensors
        gH = None
        if ctx.needs_input_grad[0]:
            kw = {k: v for k, v in ctx.opts.items() if k not in ("spin", "sweep", "ckpt_interval")}
            gH, _, _, _ = susceptibility(H, gD.contiguous(), ctx.nocc, want_density=False, sweep="adjoint",
                                         ckpt_interval=ctx.ckpt, spin=1.0, **kw)
        return gH, None, None, None


def density(H, nocc: int, *, ckpt_interval: int = 8, **opts):
    """D(H) with autograd support; `opts` are the options of sp2_density
    (precision, bounds, max_iter, ...)."""
    return SP2Density.apply(H, nocc, ckpt_interval, opts)


def observable_gradients(H, A, nocc: int, *, ckpt_interval: int = 8, spin: float = 2.0, **opts):
    """chi_k = s dTr[A_k D]/dH for a stack of observables A (nobs, n, n) in one
    backward sweep (the batched form of density(...).backward).  Returns
    (chi, D, a0, info) like susceptibility()."""
    return susceptibility(H, A, nocc, sweep="adjoint", ckpt_interval=ckpt_interval, spin=spin, **opts)
