"""MI355X (gfx950) recursive density-matrix perturbation theory in its
susceptibility form (arXiv 2409.17033).

Python binding over libdmpt (include/dmpt.h).  Every numerical step runs in
the library's HIP kernels; this module only marshals torch device tensors,
the current stream and a caller-owned workspace into the C ABI.

    D, info = sp2_density(H, nocc)                              # Eq. DM0
    chi, D, a0, info = susceptibility(H, A, nocc)               # Eq. DMSuscept / DM2
    out = response(chi, H1)                                     # Eq. dual: Tr[chi H1]
"""
from __future__ import annotations

import ctypes as C

from ._lib import (BOUNDS, PRECISION, SWEEP, DMPTError, Info, Opts, SCFOpts, check, last_error,
                   load)

__all__ = ["sp2_density", "susceptibility", "response", "response_static", "make_opts", "workspace_bytes",
           "sp2_decide", "scf_response", "DMPTError", "load"]


def _torch():
    import torch
    return torch


def _check_matrix(t, n=None, name="matrix"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and tuple(t.shape[-2:]) != (n, n):
        raise ValueError(f"{name} must have trailing shape ({n}, {n}), got {tuple(t.shape)}")


def make_opts(n: int, nocc: int, *, precision: str = "fp32", bounds: str = "lanczos",
              emin: float | None = None, emax: float | None = None, lanczos_steps: int = 0,
              max_iter: int = 0, min_iter: int = -1, sweep: str = "forward",
              idem_tol: float = 0.0, project: bool | int = True, spin: float = 2.0,
              profile: bool = False, ckpt_interval: int = 0, refine: bool | int = False,
              sweep_tol: float = 0.0, stream=None) -> Opts:
    lib = load()
    o = Opts()
    lib.dmpt_opts_default(C.byref(o), n, nocc)
    o.precision = PRECISION[precision]
    o.bounds = BOUNDS[bounds]
    if bounds == "given":
        o.emin, o.emax = float(emin), float(emax)
    o.lanczos_steps = lanczos_steps
    o.max_iter = max_iter
    o.min_iter = min_iter
    o.sweep = SWEEP[sweep]
    o.idem_tol = idem_tol
    o.project = int(project)   # True -> 1; 2: the projections above the sweep's precision (split3x)
    o.spin = spin
    o.profile = 1 if profile else 0
    o.ckpt_interval = ckpt_interval
    o.refine = int(refine)   # True -> 1; 2: the correction on the regular tiles only
    o.sweep_tol = sweep_tol
    if stream is None:
        torch = _torch()
        stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
    o.stream = stream or None
    return o


def workspace_bytes(opts: Opts, nobs: int) -> int:
    return int(load().dmpt_workspace_bytes(C.byref(opts), nobs))


def _workspace(opts: Opts, nobs: int, device):
    torch = _torch()
    nbytes = workspace_bytes(opts, nobs)
    if nbytes == 0:
        check(1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    opts.workspace = ws.data_ptr()
    opts.workspace_bytes = nbytes
    return ws


def sp2_density(H, nocc: int, *, workspace=None, raise_on_error: bool = True, **kw):
    """Eq. DM0: D = theta(mu I - H).  Returns (D, info dict).

    With raise_on_error=False a NOT_CONVERGED / BOUNDS / NONFINITE status is
    reported in info["status"] and D holds the last iterate."""
    torch = _torch()
    n = H.shape[-1]
    _check_matrix(H, n, "H")
    o = make_opts(n, nocc, **kw)
    ws = _workspace(o, 0, H.device) if workspace is None else workspace
    if workspace is not None:
        o.workspace, o.workspace_bytes = ws.data_ptr(), ws.numel()
    D = torch.empty((n, n), dtype=torch.float32, device=H.device)
    info = Info()
    st = load().dmpt_sp2_density(C.c_void_p(H.data_ptr()), C.c_void_p(D.data_ptr()), C.byref(o), C.byref(info))
    _finish(st, info, raise_on_error)
    return D, info.as_dict()


def _finish(st, info, raise_on_error):
    recoverable = st in (2, 3, 4)   # NONFINITE, NOT_CONVERGED, BOUNDS: outputs written
    if st != 0 and (raise_on_error or not recoverable):
        check(st, info)


def susceptibility(H, A, nocc: int, *, want_density: bool = True, workspace=None,
                   raise_on_error: bool = True, **kw):
    """chi^A = s dTr[A D]/dH (Eq. Suscept) by Eq. DMSuscept (or Eq. DM2 with sweep='adjoint').

    A: (n, n) or (nobs, n, n).  Returns (chi, D or None, a0 [nobs], info dict).
    """
    torch = _torch()
    n = H.shape[-1]
    _check_matrix(H, n, "H")
    _check_matrix(A, n, "A")
    single = A.dim() == 2
    nobs = 1 if single else A.shape[0]
    o = make_opts(n, nocc, **kw)
    ws = _workspace(o, nobs, H.device) if workspace is None else workspace
    if workspace is not None:
        o.workspace, o.workspace_bytes = ws.data_ptr(), ws.numel()
    chi = torch.empty((nobs, n, n), dtype=torch.float32, device=H.device)
    D = torch.empty((n, n), dtype=torch.float32, device=H.device) if want_density else None
    a0 = (C.c_double * nobs)()
    info = Info()
    st = load().dmpt_susceptibility(C.c_void_p(H.data_ptr()), C.c_void_p(A.data_ptr()), nobs,
                                    C.c_void_p(chi.data_ptr()),
                                    C.c_void_p(D.data_ptr()) if D is not None else None,
                                    a0, C.byref(o), C.byref(info))
    _finish(st, info, raise_on_error)
    return (chi[0] if single else chi), D, list(a0), info.as_dict()


def susceptibility_nonorth(H, Z, A, nocc: int, *, raise_on_error: bool = True, **kw):
    """Sec. V.A: the susceptibility in a non-orthonormal basis with inverse
    factor Z (Z^T S Z = I).  A: (n, n) or (nobs, n, n).  Returns
    (chi_perp, chi_ao, D, a0 [nobs], info dict): chi_perp is the dual of
    H_perp = Z^T H Z, chi_ao = Z chi_perp Z^T the dual of H at fixed S, D the
    atomic-orbital density matrix Z D_perp Z^T."""
    torch = _torch()
    n = H.shape[-1]
    _check_matrix(H, n, "H")
    _check_matrix(Z, n, "Z")
    _check_matrix(A, n, "A")
    single = A.dim() == 2
    nobs = 1 if single else A.shape[0]
    o = make_opts(n, nocc, **kw)
    lib = load()
    nbytes = int(lib.dmpt_nonorth_workspace_bytes(C.byref(o), nobs))
    if nbytes == 0:
        check(1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=H.device)
    o.workspace, o.workspace_bytes = ws.data_ptr(), nbytes
    chi_p = torch.empty((nobs, n, n), dtype=torch.float32, device=H.device)
    chi_ao = torch.empty((nobs, n, n), dtype=torch.float32, device=H.device)
    D = torch.empty((n, n), dtype=torch.float32, device=H.device)
    a0 = (C.c_double * nobs)()
    info = Info()
    st = lib.dmpt_susceptibility_nonorth(C.c_void_p(H.data_ptr()), C.c_void_p(Z.data_ptr()),
                                         C.c_void_p(A.data_ptr()), nobs, C.c_void_p(chi_p.data_ptr()),
                                         C.c_void_p(chi_ao.data_ptr()), C.c_void_p(D.data_ptr()), a0,
                                         C.byref(o), C.byref(info))
    _finish(st, info, raise_on_error)
    if single:
        chi_p, chi_ao = chi_p[0], chi_ao[0]
    return chi_p, chi_ao, D, list(a0), info.as_dict()


def susceptibility_fermi(H, A, nocc: int, kt: float, *, canonical: bool = True, mu: float = float("nan"),
                         doublings: int = 0, newton_max: int = 0, count_tol: float = 0.0,
                         raise_on_error: bool = True, **kw):
    """Sec. V.B: D = f(H) (Fermi function at k_B T_e = kt) and the
    temperature-dependent susceptibility chi = s d/dlambda f(H + lambda (A + mu_1 I))
    by the recursive doubling expansion (dmpt_susceptibility_fermi).  A:
    (n, n), (nobs, n, n) or None.  Returns (chi or None, D, a0 [nobs], info dict)."""
    torch = _torch()
    from ._lib import FermiInfo, FermiOpts
    n = H.shape[-1]
    _check_matrix(H, n, "H")
    nobs = 0
    single = False
    if A is not None:
        _check_matrix(A, n, "A")
        single = A.dim() == 2
        nobs = 1 if single else A.shape[0]
    o = make_opts(n, nocc, **kw)
    f = FermiOpts(kt=kt, mu=mu, count_tol=count_tol, canonical=1 if canonical else 0, doublings=doublings,
                  newton_max=newton_max)
    lib = load()
    nbytes = int(lib.dmpt_fermi_workspace_bytes(C.byref(o), C.byref(f), nobs))
    if nbytes == 0:
        check(1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=H.device)
    o.workspace, o.workspace_bytes = ws.data_ptr(), nbytes
    chi = torch.empty((max(nobs, 1), n, n), dtype=torch.float32, device=H.device) if nobs else None
    D = torch.empty((n, n), dtype=torch.float32, device=H.device)
    a0 = (C.c_double * max(nobs, 1))()
    info = FermiInfo()
    st = lib.dmpt_susceptibility_fermi(C.c_void_p(H.data_ptr()), C.c_void_p(A.data_ptr()) if nobs else None, nobs,
                                       C.c_void_p(chi.data_ptr()) if nobs else None, C.c_void_p(D.data_ptr()), a0,
                                       C.byref(f), C.byref(o), C.byref(info))
    if st != 0 and (raise_on_error or st != 3):
        check(st)
    if chi is not None and single:
        chi = chi[0]
    return chi, D, list(a0[:nobs]), info.as_dict(nobs)


def response(chi, H1, *, stream=None):
    """Eq. dual: out[k, p] = Tr[chi_k H1_p] (FP64).  chi: (n,n)/(K,n,n); H1: (n,n)/(P,n,n)."""
    torch = _torch()
    n = chi.shape[-1]
    _check_matrix(chi, n, "chi")
    _check_matrix(H1, n, "H1")
    k = 1 if chi.dim() == 2 else chi.shape[0]
    p = 1 if H1.dim() == 2 else H1.shape[0]
    lib = load()
    nbytes = int(lib.dmpt_response_workspace_bytes(k, p, n))
    if nbytes == 0:
        check(1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=chi.device)
    out = (C.c_double * (k * p))()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st = lib.dmpt_response(C.c_void_p(chi.data_ptr()), k, C.c_void_p(H1.data_ptr()), p, n, out,
                           C.c_void_p(stream) if stream else None, C.c_void_p(ws.data_ptr()), nbytes)
    check(st)
    import numpy as np
    return np.array(out[:], dtype=np.float64).reshape(k, p)


def response_static(chi, H1, *, stream=None):
    """dmpt_response_static: Tr[chi_k H1_p] like response(), with the
    library's own device scratch instead of a workspace (no allocation in
    the call; calls that overlap on one device race on that scratch)."""
    torch = _torch()
    n = chi.shape[-1]
    _check_matrix(chi, n, "chi")
    _check_matrix(H1, n, "H1")
    k = 1 if chi.dim() == 2 else chi.shape[0]
    p = 1 if H1.dim() == 2 else H1.shape[0]
    out = (C.c_double * (k * p))()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    check(load().dmpt_response_static(C.c_void_p(chi.data_ptr()), k, C.c_void_p(H1.data_ptr()), p, n, out,
                                      C.c_void_p(stream) if stream else None))
    import numpy as np
    return np.array(out[:], dtype=np.float64).reshape(k, p)


def sp2_decide(tr, sq, eps, eps_prev1, eps_prev2, eps_prev3, steps, n, nocc, min_iter=10, idem_tol=0.0,
               precision: str = "fp32") -> int:
    """Host mirror of the device step controller (dmpt_sp2_decide in include/dmpt.h):
    -3 bounds violation, 0 stop, else sigma_n (+1 / -1) for iterate X_n, from
    eps_n and eps_{n-1}, eps_{n-2}, eps_{n-3}, for the product precision."""
    return int(load().dmpt_sp2_decide(tr, sq, eps, eps_prev1, eps_prev2, eps_prev3, steps, n, nocc,
                                      min_iter, idem_tol, PRECISION[precision]))


def scf_response(H0, U, A, nocc: int, *, mixer: str = "linear", max_iter: int = 200, mix: float = 0.3,
                 tol: float = 1e-6, anderson_depth: int = 5, net=None, record: bool = False,
                 raise_on_error: bool = True, **kw):
    """Eq. CP_SCF: self-consistent chi = s chi', chi' = L[A + G(chi')], G(X) = diag(U s diag X).

    mixer: "linear" (c_mix = mix), "anderson", "learned" (net: a mixer.Mixer) or
    "learned_anderson" (Anderson extrapolation with the network as preconditioner).
    Returns (chi, scf_info dict, info dict of the SP2 recursion); with
    record=True also (v, r) of every accepted state, each (states, n).
    """
    torch = _torch()
    from ._lib import MIXER, SCFInfo, SCFOpts
    n = H0.shape[-1]
    _check_matrix(H0, n, "H0")
    _check_matrix(A, n, "A")
    o = make_opts(n, nocc, sweep="adjoint", **kw)
    sopt = SCFOpts(max_iter=max_iter, mixer=MIXER[mixer], mix=mix, tol=tol, anderson_depth=anderson_depth)
    if mixer in ("learned", "learned_anderson"):
        if net is None:
            raise ValueError("the learned mixer needs net=Mixer(...)")
        sopt.mlp_hidden, sopt.mlp_window = net.hidden, net.window
        sopt.mlp_params = net.params.data_ptr()
    rec_v = rec_r = None
    if record:
        rec_v = torch.zeros((max_iter, n), dtype=torch.float32, device=H0.device)
        rec_r = torch.zeros((max_iter, n), dtype=torch.float32, device=H0.device)
        sopt.record_v, sopt.record_r = rec_v.data_ptr(), rec_r.data_ptr()
    lib = load()
    nbytes = int(lib.dmpt_scf_workspace_bytes(C.byref(o), C.byref(sopt)))
    if nbytes == 0:
        check(1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=H0.device)
    o.workspace, o.workspace_bytes = ws.data_ptr(), nbytes
    chi = torch.empty((n, n), dtype=torch.float32, device=H0.device)
    info, sinfo = Info(), SCFInfo()
    st = lib.dmpt_scf_response(C.c_void_p(H0.data_ptr()), C.c_void_p(U.data_ptr()), C.c_void_p(A.data_ptr()),
                               C.c_void_p(chi.data_ptr()), C.byref(sopt), C.byref(o), C.byref(info),
                               C.byref(sinfo))
    if st != 0 and (raise_on_error or st != 3):
        check(st, info)
    out = (chi, sinfo.as_dict(), info.as_dict())
    if record:
        out = out + (rec_v[:sinfo.states], rec_r[:sinfo.states])
    return out
