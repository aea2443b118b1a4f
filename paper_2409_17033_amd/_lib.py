"""ctypes declarations of the libdmpt C ABI (include/dmpt.h).

Loading fails loudly: there is no CPU fallback for any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmpt.so")

DMPT_MAX_STEPS = 255

STATUS = {
    0: "DMPT_OK",
    1: "DMPT_ERR_ARG",
    2: "DMPT_ERR_NONFINITE",
    3: "DMPT_ERR_NOT_CONVERGED",
    4: "DMPT_ERR_BOUNDS",
    5: "DMPT_ERR_DEVICE",
    6: "DMPT_ERR_WORKSPACE",
    7: "DMPT_ERR_UNSUPPORTED",
}

ABI_VERSION = 8   # DMPT_ABI_VERSION of include/dmpt.h this binding is written against
PRECISION = {"fp32": 0, "split_bf16": 1, "split3_bf16": 2, "bf16": 3, "split3x_bf16": 4, "split_fp16": 5}
BOUNDS = {"lanczos": 0, "gershgorin": 1, "given": 2}
SWEEP = {"forward": 0, "adjoint": 1}

EXPORTS = [
    "dmpt_abi_version", "dmpt_opts_default", "dmpt_workspace_bytes", "dmpt_sp2_density",
    "dmpt_susceptibility", "dmpt_response_workspace_bytes", "dmpt_response", "dmpt_response_static",
    "dmpt_scf_response", "dmpt_scf_workspace_bytes", "dmpt_mixer_param_count", "dmpt_mixer_workspace_bytes",
    "dmpt_mixer_init", "dmpt_mixer_forward", "dmpt_mixer_loss_grad", "dmpt_mixer_train",
    "dmpt_mixer_rows_workspace_bytes", "dmpt_mixer_pairs", "dmpt_mixer_shuffle",
    "dmpt_nonorth_workspace_bytes", "dmpt_susceptibility_nonorth",
    "dmpt_fermi_workspace_bytes", "dmpt_susceptibility_fermi",
    "dmpt_sp2_decide", "dmpt_status_string", "dmpt_last_error",
]


class Opts(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("nocc", C.c_int32), ("precision", C.c_int32), ("bounds", C.c_int32),
        ("emin", C.c_double), ("emax", C.c_double),
        ("lanczos_steps", C.c_int32), ("max_iter", C.c_int32), ("min_iter", C.c_int32),
        ("sweep", C.c_int32),
        ("idem_tol", C.c_double),
        ("project", C.c_int32), ("profile", C.c_int32),
        ("ckpt_interval", C.c_int32), ("refine", C.c_int32),
        ("sweep_tol", C.c_double),
        ("spin", C.c_double),
        ("stream", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
    ]


class Info(C.Structure):
    _fields_ = [
        ("m", C.c_int32), ("status", C.c_int32),
        ("emin", C.c_double), ("emax", C.c_double), ("beta", C.c_double),
        ("trace_d", C.c_double), ("idem_err", C.c_double), ("elapsed_ms", C.c_double),
        ("sigma", C.c_int8 * (DMPT_MAX_STEPS + 1)),
        ("trace_x", C.c_double * (DMPT_MAX_STEPS + 1)),
        ("sqnorm_x", C.c_double * (DMPT_MAX_STEPS + 1)),
        ("idem_x", C.c_double * (DMPT_MAX_STEPS + 1)),
        ("bounds_ms", C.c_double), ("step_ms", C.c_double), ("project_ms", C.c_double),
        ("output_ms", C.c_double), ("step_launches", C.c_int32), ("tile", C.c_int32),
        ("refine_ms", C.c_double),
        ("sweep_steps", C.c_int32), ("correction_steps", C.c_int32),
        ("split_tiles", C.c_int32), ("split_tiles_sweep", C.c_int32),
    ]

    def as_dict(self) -> dict:
        m = self.m
        return {
            "m": m, "status": STATUS.get(self.status, self.status), "emin": self.emin,
            "emax": self.emax, "beta": self.beta, "trace_d": self.trace_d,
            "idem_err": self.idem_err, "elapsed_ms": self.elapsed_ms,
            "sigma": list(self.sigma[:m]), "sigma_next": int(self.sigma[m]) if m < len(self.sigma) else 0,
            "trace_x": list(self.trace_x[:m + 1]),
            "sqnorm_x": list(self.sqnorm_x[:m + 1]),
            "idem_x": list(self.idem_x[:m + 1]),
            "bounds_ms": self.bounds_ms, "step_ms": self.step_ms, "project_ms": self.project_ms,
            "output_ms": self.output_ms, "step_launches": self.step_launches, "tile": self.tile,
            "refine_ms": self.refine_ms, "sweep_steps": self.sweep_steps,
            "correction_steps": self.correction_steps, "split_tiles": self.split_tiles,
            "split_tiles_sweep": self.split_tiles_sweep,
        }


MIXER = {"linear": 0, "anderson": 1, "learned": 2, "learned_anderson": 3}
DMPT_MAX_SCF = 1024


class SCFOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("mixer", C.c_int32), ("mix", C.c_double), ("tol", C.c_double),
                ("anderson_depth", C.c_int32), ("mlp_hidden", C.c_int32), ("mlp_window", C.c_int32),
                ("reserved", C.c_int32), ("mlp_params", C.c_void_p),
                ("record_v", C.c_void_p), ("record_r", C.c_void_p)]


class SCFInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rejected", C.c_int32),
                ("states", C.c_int32), ("residual", C.c_double * DMPT_MAX_SCF)]

    def as_dict(self) -> dict:
        return {"iters": self.iters, "converged": bool(self.converged), "rejected": self.rejected,
                "states": self.states, "residual": list(self.residual[:self.states])}


class FermiOpts(C.Structure):
    _fields_ = [("kt", C.c_double), ("mu", C.c_double), ("count_tol", C.c_double), ("canonical", C.c_int32),
                ("doublings", C.c_int32), ("newton_max", C.c_int32), ("reserved", C.c_int32)]


class FermiInfo(C.Structure):
    _fields_ = [("mu", C.c_double), ("trace_d", C.c_double), ("emin", C.c_double), ("emax", C.c_double),
                ("doublings", C.c_int32), ("newton", C.c_int32), ("products", C.c_int32), ("reserved", C.c_int32),
                ("mu1", C.c_double * 64), ("elapsed_ms", C.c_double)]

    def as_dict(self, nobs: int = 0) -> dict:
        return {"mu": self.mu, "trace_d": self.trace_d, "emin": self.emin, "emax": self.emax,
                "doublings": self.doublings, "newton": self.newton, "products": self.products,
                "mu1": list(self.mu1[:nobs]), "elapsed_ms": self.elapsed_ms}


class DMPTError(RuntimeError):
    def __init__(self, status: int, message: str, info: dict | None = None):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        self.info = info


_lib = None


def load() -> C.CDLL:
    """Load libdmpt.so (built in-tree by paper_2409_17033_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2409_17033_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, I32, D, SZ = C.c_void_p, C.c_int32, C.c_double, C.c_size_t
    lib.dmpt_abi_version.restype = I32
    if lib.dmpt_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {lib.dmpt_abi_version()}, this binding expects "
                          f"{ABI_VERSION}: rebuild it with `python -m paper_2409_17033_amd.build`")
    lib.dmpt_opts_default.argtypes = [C.POINTER(Opts), I32, I32]
    lib.dmpt_opts_default.restype = None
    lib.dmpt_workspace_bytes.argtypes = [C.POINTER(Opts), I32]
    lib.dmpt_workspace_bytes.restype = SZ
    lib.dmpt_sp2_density.argtypes = [P, P, C.POINTER(Opts), C.POINTER(Info)]
    lib.dmpt_sp2_density.restype = C.c_int
    lib.dmpt_susceptibility.argtypes = [P, P, I32, P, P, C.POINTER(D), C.POINTER(Opts), C.POINTER(Info)]
    lib.dmpt_susceptibility.restype = C.c_int
    lib.dmpt_nonorth_workspace_bytes.argtypes = [C.POINTER(Opts), I32]
    lib.dmpt_nonorth_workspace_bytes.restype = C.c_size_t
    lib.dmpt_susceptibility_nonorth.argtypes = [P, P, P, I32, P, P, P, C.POINTER(D), C.POINTER(Opts),
                                                C.POINTER(Info)]
    lib.dmpt_susceptibility_nonorth.restype = C.c_int
    lib.dmpt_fermi_workspace_bytes.argtypes = [C.POINTER(Opts), C.POINTER(FermiOpts), I32]
    lib.dmpt_fermi_workspace_bytes.restype = C.c_size_t
    lib.dmpt_susceptibility_fermi.argtypes = [P, P, I32, P, P, C.POINTER(D), C.POINTER(FermiOpts), C.POINTER(Opts),
                                              C.POINTER(FermiInfo)]
    lib.dmpt_susceptibility_fermi.restype = C.c_int
    lib.dmpt_response_workspace_bytes.argtypes = [I32, I32, I32]
    lib.dmpt_response_workspace_bytes.restype = SZ
    lib.dmpt_response.argtypes = [P, I32, P, I32, I32, C.POINTER(D), P, P, SZ]
    lib.dmpt_response.restype = C.c_int
    lib.dmpt_response_static.argtypes = [P, I32, P, I32, I32, C.POINTER(D), P]
    lib.dmpt_response_static.restype = C.c_int
    lib.dmpt_scf_response.argtypes = [P, P, P, P, C.POINTER(SCFOpts), C.POINTER(Opts), C.POINTER(Info),
                                      C.POINTER(SCFInfo)]
    lib.dmpt_scf_response.restype = C.c_int
    lib.dmpt_scf_workspace_bytes.argtypes = [C.POINTER(Opts), C.POINTER(SCFOpts)]
    lib.dmpt_scf_workspace_bytes.restype = SZ
    lib.dmpt_mixer_param_count.argtypes = [I32, I32]
    lib.dmpt_mixer_param_count.restype = SZ
    lib.dmpt_mixer_workspace_bytes.argtypes = [I32, I32, I32, I32]
    lib.dmpt_mixer_workspace_bytes.restype = SZ
    lib.dmpt_mixer_init.argtypes = [P, P, I32, I32, C.c_uint64, P]
    lib.dmpt_mixer_init.restype = C.c_int
    lib.dmpt_mixer_forward.argtypes = [P, I32, I32, P, P, I32, P, I32, P, P, P, SZ]
    lib.dmpt_mixer_forward.restype = C.c_int
    lib.dmpt_mixer_loss_grad.argtypes = [P, I32, I32, P, P, I32, P, P, I32, P, C.POINTER(D), P, P, SZ]
    lib.dmpt_mixer_loss_grad.restype = C.c_int
    lib.dmpt_mixer_train.argtypes = [P, P, P, P, I32, I32, P, P, I32, P, P, I32, I32, I32, D, C.POINTER(D), P, P,
                                     SZ]
    lib.dmpt_mixer_train.restype = C.c_int
    lib.dmpt_mixer_rows_workspace_bytes.argtypes = [I32]
    lib.dmpt_mixer_rows_workspace_bytes.restype = SZ
    lib.dmpt_mixer_pairs.argtypes = [P, P, C.POINTER(D), I32, I32, P, D, D, I32, P, P, I32, C.POINTER(I32), P, P,
                                     SZ]
    lib.dmpt_mixer_pairs.restype = C.c_int
    lib.dmpt_mixer_shuffle.argtypes = [P, P, I32, I32, C.c_uint64, P, P, P, P, SZ]
    lib.dmpt_mixer_shuffle.restype = C.c_int
    lib.dmpt_sp2_decide.argtypes = [D, D, D, D, D, D, I32, I32, D, I32, D, I32]
    lib.dmpt_sp2_decide.restype = I32
    lib.dmpt_status_string.argtypes = [C.c_int]
    lib.dmpt_status_string.restype = C.c_char_p
    lib.dmpt_last_error.argtypes = []
    lib.dmpt_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    return load().dmpt_last_error().decode()


def check(status: int, info: Info | None = None) -> None:
    if status != 0:
        raise DMPTError(status, last_error(), info.as_dict() if info is not None else None)
