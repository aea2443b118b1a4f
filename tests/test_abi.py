"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/dmpt.h, the ctypes layouts match, argument validation
fails before any HIP call, and the host mirror of the step controller agrees
with the oracle's sigma / stop rule."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmpt.h")
LIB = os.path.join(ROOT, "paper_2409_17033_amd", "libdmpt.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdmpt.so not built")


@pytest.fixture(scope="module")
def lib():
    from paper_2409_17033_amd import _lib
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmpt_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_no_undeclared_c_exports():
    """Every unmangled (C) symbol the library exports is a declared entry
    point: the runtime's helpers have internal linkage."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    syms = [line.split()[-1] for line in out.splitlines() if line.split()[-2:-1] and line.split()[-2] in "TtWw"]
    c_syms = [x for x in syms if not x.startswith("_Z")]
    declared = set(declared_functions())
    assert c_syms and not [x for x in c_syms if x not in declared], [x for x in c_syms if x not in declared]


def test_abi_version(lib):
    assert lib.dmpt_abi_version() == 8


def test_struct_layouts():
    from paper_2409_17033_amd._lib import Info, Opts
    # sizes follow from the C declarations with natural alignment
    assert C.sizeof(Opts) == 112
    assert Opts.sweep_tol.offset == 72
    assert Opts.spin.offset == 80 and Opts.workspace_bytes.offset == 104
    assert Opts.ckpt_interval.offset == 64
    assert Info.sigma.offset == 56
    assert C.sizeof(Info) == 56 + 256 + 3 * 256 * 8 + 4 * 8 + 2 * 4 + 8 + 4 * 4
    assert Info.idem_x.offset == 56 + 256 + 2 * 256 * 8
    assert Opts.profile.offset == 60


def test_opts_default(lib):
    from paper_2409_17033_amd._lib import Opts
    o = Opts()
    lib.dmpt_opts_default(C.byref(o), 100, 40)
    assert (o.n, o.nocc, o.precision, o.bounds, o.max_iter, o.min_iter, o.project, o.spin) == \
        (100, 40, 0, 0, 100, 10, 1, 2.0)


def _opts(lib, n=64, nocc=32, **kw):
    from paper_2409_17033_amd._lib import Opts
    o = Opts()
    lib.dmpt_opts_default(C.byref(o), n, nocc)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_checkpoint_workspace(lib):
    """Adjoint with checkpoints every k steps: 2 working + ceil slots + k - 1 ring
    instead of max_iter + 3 slots."""
    full = _opts(lib, 1000, 500, sweep=1)
    w_full = lib.dmpt_workspace_bytes(C.byref(full), 1)
    slot = 1024 * 1024 * 4 + 2304   # FP32 master + metadata (8 B + 256 FP64 partials, 256-aligned)
    for k in (1, 4, 8, 16):
        ck = _opts(lib, 1000, 500, sweep=1, ckpt_interval=k)
        w = lib.dmpt_workspace_bytes(C.byref(ck), 1)
        nslots = 2 + (100 + 1) // k + 1 + (k - 1)
        assert w_full - w == (103 - nslots) * slot, k
    bad = _opts(lib, 1000, 500, sweep=1, ckpt_interval=-1)
    assert lib.dmpt_workspace_bytes(C.byref(bad), 1) == 0
    bad = _opts(lib, 1000, 500, refine=3)
    assert lib.dmpt_workspace_bytes(C.byref(bad), 1) == 0
    # the residual correction needs the forward sweep with the projection
    bad = _opts(lib, 1000, 500, refine=1, sweep=1)
    assert lib.dmpt_workspace_bytes(C.byref(bad), 1) == 0
    bad = _opts(lib, 1000, 500, refine=1, project=0)
    assert lib.dmpt_workspace_bytes(C.byref(bad), 1) == 0
    # it adds its own buffers to the plain solve's workspace
    plain = _opts(lib, 1000, 500, precision=1)
    ref = _opts(lib, 1000, 500, precision=1, refine=1)
    assert lib.dmpt_workspace_bytes(C.byref(ref), 1) > lib.dmpt_workspace_bytes(C.byref(plain), 1)


def test_sweep_tol_validation(lib):
    """The sweep stop is an option of the residual correction: without it,
    or outside [0, 1/4), the options are refused before any device work."""
    ok = _opts(lib, 1000, 500, precision=4, refine=1, sweep_tol=1e-4)
    assert lib.dmpt_workspace_bytes(C.byref(ok), 1) > 0
    for tol, refine in ((1e-4, 0), (-1e-4, 1), (0.25, 1), (float("nan"), 1), (float("inf"), 1)):
        bad = _opts(lib, 1000, 500, precision=4, refine=refine, sweep_tol=tol)
        assert lib.dmpt_workspace_bytes(C.byref(bad), 1) == 0, (tol, refine)
        assert lib.dmpt_susceptibility(FAKE, FAKE, 1, FAKE, None, None, C.byref(bad), None) == 1
        assert b"sweep_tol" in lib.dmpt_last_error()


def test_project_validation(lib):
    """project = 2 (the projections above the sweep's precision) exists for
    the three-term-X^2 option with the correction only; it needs no more
    workspace than project = 1 (it reuses the free Y slot and the main list's
    buffer); other values are refused before any device work."""
    ok = _opts(lib, 1000, 500, precision=4, refine=1, project=2)
    base = _opts(lib, 1000, 500, precision=4, refine=1, project=1)
    assert lib.dmpt_workspace_bytes(C.byref(ok), 2) == lib.dmpt_workspace_bytes(C.byref(base), 2) > 0
    for prec, refine, project in ((4, 0, 2), (2, 1, 2), (5, 1, 2), (0, 1, 2), (4, 1, 3), (4, 1, -1)):
        bad = _opts(lib, 1000, 500, precision=prec, refine=refine, project=project)
        assert lib.dmpt_workspace_bytes(C.byref(bad), 1) == 0, (prec, refine, project)
        assert lib.dmpt_susceptibility(FAKE, FAKE, 1, FAKE, None, None, C.byref(bad), None) == 1
        assert b"project" in lib.dmpt_last_error()


def test_workspace_bytes(lib):
    o = _opts(lib, 1000, 500)
    w0 = lib.dmpt_workspace_bytes(C.byref(o), 0)
    w1 = lib.dmpt_workspace_bytes(C.byref(o), 1)
    w2 = lib.dmpt_workspace_bytes(C.byref(o), 2)
    n_pad = 1024
    assert w0 > 2 * n_pad * n_pad * 4          # two FP32 iterates
    assert w2 - w1 == w1 - w0 or w2 > w1 > w0
    o.precision = 1                             # split adds the operand copy
    assert lib.dmpt_workspace_bytes(C.byref(o), 1) > w1
    o.sweep = 1                                 # adjoint stores every X_n
    assert lib.dmpt_workspace_bytes(C.byref(o), 1) > 50 * n_pad * n_pad * 8
    bad = _opts(lib, 0, 0)
    assert lib.dmpt_workspace_bytes(C.byref(bad), 1) == 0


FAKE = C.c_void_p(0x1000)   # never dereferenced: validation fails first


@pytest.mark.parametrize("field,value", [
    ("n", 0), ("n", 70000), ("nocc", -1), ("nocc", 65), ("precision", 9), ("bounds", 7),
    ("max_iter", 300), ("lanczos_steps", -2), ("sweep", 5), ("idem_tol", -1.0),
    ("spin", float("nan")), ("project", 3),
])
def test_invalid_options_rejected_before_device(lib, field, value):
    o = _opts(lib, **{field: value})
    from paper_2409_17033_amd._lib import Info
    info = Info()
    assert lib.dmpt_sp2_density(FAKE, FAKE, C.byref(o), C.byref(info)) == 1
    assert lib.dmpt_last_error()


def test_null_pointers_and_workspace(lib):
    o = _opts(lib)
    assert lib.dmpt_sp2_density(None, FAKE, C.byref(o), None) == 1
    assert lib.dmpt_sp2_density(FAKE, None, C.byref(o), None) == 1
    assert lib.dmpt_sp2_density(FAKE, FAKE, None, None) == 1
    a0 = (C.c_double * 1)()
    assert lib.dmpt_susceptibility(FAKE, None, 1, FAKE, None, a0, C.byref(o), None) == 1
    assert lib.dmpt_susceptibility(FAKE, FAKE, 0, FAKE, None, a0, C.byref(o), None) == 1
    # valid arguments but no workspace -> DMPT_ERR_WORKSPACE
    assert lib.dmpt_sp2_density(FAKE, FAKE, C.byref(o), None) == 6
    o.workspace = 0x2000
    o.workspace_bytes = 16
    assert lib.dmpt_sp2_density(FAKE, FAKE, C.byref(o), None) == 6
    assert b"need" in lib.dmpt_last_error()


def test_given_bounds_validation(lib):
    o = _opts(lib, bounds=2, emin=1.0, emax=1.0)
    assert lib.dmpt_sp2_density(FAKE, FAKE, C.byref(o), None) == 1


@pytest.mark.parametrize("prec", [2, 4])
def test_split3_accepted(lib, prec):
    o = _opts(lib, precision=prec)
    assert lib.dmpt_workspace_bytes(C.byref(o), 1) > 0
    assert lib.dmpt_sp2_density(FAKE, FAKE, C.byref(o), None) == 6   # passes validation


def test_split3x_workspace_adds_two_term_copies(lib):
    """The mixed mode keeps the three-term copy of every matrix slot plus a
    two-term copy (4 bytes per element): split-3's workspace plus 4 n_pad^2
    bytes for each of the 2 X slots and 2 x nobs Y slots."""
    a, b = _opts(lib, 1000, 500, precision=2), _opts(lib, 1000, 500, precision=4)
    n_pad, nobs = 1024, 2
    extra = (2 + 2 * nobs) * 4 * n_pad * n_pad
    assert lib.dmpt_workspace_bytes(C.byref(b), nobs) - lib.dmpt_workspace_bytes(C.byref(a), nobs) == extra


def test_response_validation(lib):
    out = (C.c_double * 4)()
    assert lib.dmpt_response(None, 1, FAKE, 1, 8, out, None, FAKE, 1 << 20) == 1
    assert lib.dmpt_response(FAKE, 0, FAKE, 1, 8, out, None, FAKE, 1 << 20) == 1
    assert lib.dmpt_response(FAKE, 1, FAKE, 0, 8, out, None, FAKE, 1 << 20) == 1
    assert lib.dmpt_response(FAKE, 2048, FAKE, 1024, 8, out, None, FAKE, 1 << 20) == 1   # > 2^20 outputs
    assert lib.dmpt_response(FAKE, 1, FAKE, 1, 0, out, None, FAKE, 1 << 20) == 1
    assert lib.dmpt_response(FAKE, 1, FAKE, 1, 8, out, None, None, 0) == 6
    assert lib.dmpt_response(FAKE, 16, FAKE, 32, 8, out, None, FAKE, 64) == 6   # too small
    assert lib.dmpt_response_workspace_bytes(1, 8, 8192) > 0
    # groups of 8 x 64: partials sized for one group, outputs for all
    assert lib.dmpt_response_workspace_bytes(16, 32, 8192) > lib.dmpt_response_workspace_bytes(8, 32, 8192)


def test_scf_response_validation(lib):
    """Argument checks of dmpt_scf_response (none reaches the device)."""
    from paper_2409_17033_amd._lib import SCFInfo, SCFOpts
    o = _opts(lib)
    s = SCFOpts(max_iter=10, mix=0.3, tol=1e-6)
    si = SCFInfo()
    assert lib.dmpt_scf_response(FAKE, FAKE, FAKE, FAKE, C.byref(s), C.byref(o), None, C.byref(si)) == 6
    assert lib.dmpt_scf_response(FAKE, None, FAKE, FAKE, C.byref(s), C.byref(o), None, None) == 1
    for field, value in (("mix", 0.0), ("mix", 1.5), ("tol", 0.0), ("max_iter", 0), ("max_iter", 5000),
                         ("mixer", 3)):
        bad = SCFOpts(max_iter=10, mix=0.3, tol=1e-6)
        setattr(bad, field, value)
        assert lib.dmpt_scf_response(FAKE, FAKE, FAKE, FAKE, C.byref(bad), C.byref(o), None, None) == 1, field
        assert lib.dmpt_scf_workspace_bytes(C.byref(o), C.byref(bad)) == 0
    andersen = SCFOpts(max_iter=10, mixer=1, mix=0.3, tol=1e-6, anderson_depth=0)
    assert lib.dmpt_scf_response(FAKE, FAKE, FAKE, FAKE, C.byref(andersen), C.byref(o), None, None) == 1
    learned = SCFOpts(max_iter=10, mixer=2, mix=0.3, tol=1e-6, mlp_hidden=16, mlp_window=4)   # no parameters
    assert lib.dmpt_scf_response(FAKE, FAKE, FAKE, FAKE, C.byref(learned), C.byref(o), None, None) == 1


def test_scf_workspace_covers_the_adjoint_solve(lib):
    from paper_2409_17033_amd._lib import SCFOpts
    o = _opts(lib, 1000, 500)
    s = SCFOpts(max_iter=10, mix=0.3, tol=1e-6)
    o.sweep = 1
    adj = lib.dmpt_workspace_bytes(C.byref(o), 1)
    o.sweep = 0
    ws = lib.dmpt_scf_workspace_bytes(C.byref(o), C.byref(s))
    assert ws >= adj + 4 * 1000 * 1000 * 4       # adjoint solve + chi_A, two chi_W, diag(U s v)
    s.mixer, s.anderson_depth = 1, 8
    assert lib.dmpt_scf_workspace_bytes(C.byref(o), C.byref(s)) >= ws + 2 * 8 * 1000 * 8


def test_mixer_sizes(lib):
    k = 4 * 32 + 3
    assert lib.dmpt_mixer_param_count(32, 256) == 256 * k + 2 * 256 + 1
    assert lib.dmpt_mixer_param_count(-1, 256) == 0
    assert lib.dmpt_mixer_workspace_bytes(1024, 32, 256, 64) > 64 * 1024 * (k + 2 * 256) * 4
    assert lib.dmpt_mixer_workspace_bytes(1024, 32, 0, 64) == 0
    out = (C.c_double * 1)()
    assert lib.dmpt_mixer_forward(FAKE, 2, 4, FAKE, FAKE, 8, FAKE, 2, FAKE, None, None, 0) == 6
    assert lib.dmpt_mixer_forward(None, 2, 4, FAKE, FAKE, 8, FAKE, 2, FAKE, None, FAKE, 1 << 20) == 1
    assert lib.dmpt_mixer_forward(FAKE, 2, 4, FAKE, None, 8, FAKE, 2, FAKE, None, FAKE, 1 << 20) == 1   # no E
    assert lib.dmpt_mixer_train(FAKE, FAKE, FAKE, FAKE, 2, 4, FAKE, FAKE, 8, FAKE, FAKE, 1, 2, 10, 1e-3, out, None,
                                FAKE, 1 << 20) == 1     # npairs < batch


def test_mixer_pairs_validation(lib):
    """Argument checks of the mixer's pair labelling and shuffle run before any device call."""
    assert lib.dmpt_mixer_rows_workspace_bytes(0) == 0
    assert lib.dmpt_mixer_rows_workspace_bytes(10) >= 40
    res = (C.c_double * 4)(1.0, 1.0, 1.0, 1.0)
    cnt = C.c_int32(0)
    p = C.c_void_p(16)
    assert lib.dmpt_mixer_pairs(None, p, res, 4, 8, p, 0.3, 1e-5, 0, p, p, 4, C.byref(cnt), None, p, 64) == 1
    assert lib.dmpt_mixer_pairs(p, p, res, 0, 8, p, 0.3, 1e-5, 0, p, p, 4, C.byref(cnt), None, p, 64) == 1
    assert lib.dmpt_mixer_pairs(p, p, res, 4, 8, p, 0.3, 1e-5, 2, p, p, 4, C.byref(cnt), None, p, 64) == 1
    assert lib.dmpt_mixer_pairs(p, p, res, 4, 8, p, 0.3, 1e-5, 0, p, p, 4, C.byref(cnt), None, p, 8) == 6
    assert lib.dmpt_mixer_pairs(p, p, res, 4, 8, p, 0.3, 1e-5, 0, p, p, 3, C.byref(cnt), None, p, 256) == 1
    assert lib.dmpt_mixer_shuffle(p, p, 4, 8, 1, p, p, None, p, 64) == 1     # in place
    assert lib.dmpt_mixer_shuffle(p, p, 4, 8, 1, C.c_void_p(32), C.c_void_p(48), None, None, 0) == 6


def test_response_static_refuses_before_device(lib):
    """dmpt_response_static checks its arguments and its 4 MiB scratch limit
    before any device call (the pointers here are never dereferenced)."""
    out = (C.c_double * 512)()
    p = C.c_void_p(16)
    assert lib.dmpt_response_static(None, 1, p, 1, 8, out, None) == 1
    assert lib.dmpt_response_static(p, 0, p, 1, 8, out, None) == 1
    # n = 8192: 2048 partial blocks x 8 observables x 64 perturbations = 8 MiB of partials
    assert lib.dmpt_response_static(p, 8, p, 64, 8192, out, None) == 6
    assert b"4 MiB" in lib.dmpt_last_error()
    # n = 1: the nobs x npert results alone exceed 4 MiB
    big = (C.c_double * 600000)()
    assert lib.dmpt_response_static(p, 1, p, 600000, 1, big, None) == 6


def test_status_strings(lib):
    lib.dmpt_status_string.restype = C.c_char_p
    assert lib.dmpt_status_string(0) == b"DMPT_OK"
    assert lib.dmpt_status_string(4) == b"DMPT_ERR_BOUNDS"


def test_controller_sigma_matches_oracle_rule():
    """The library's sigma choice equals the oracle's on random traces."""
    import paper_2409_17033_amd as dm
    from oracle import sp2
    rng = np.random.default_rng(0)
    for _ in range(500):
        n = int(rng.integers(2, 5000))
        nocc = float(rng.integers(1, n))
        tr = rng.uniform(0, n)
        sq = tr * rng.uniform(0.0, 1.0)
        got = dm.sp2_decide(tr, sq, 0.5, 0.0, 0.0, 0.0, 0, n, nocc, min_iter=10)
        assert got == sp2.choose_sigma(tr, sq, nocc)


def test_controller_replays_oracle_run():
    """Feed the FP64 oracle's traces and idempotency errors to the library
    controller: it must continue with the same sigma at every step and stop
    at the same M."""
    import paper_2409_17033_amd as dm
    import workloads as W
    from oracle import sp2
    for wl in (W.dense_gapped(128), W.dense_gapped(96, nocc=20, gap=0.05)):
        h = wl.H.astype(np.float64)
        _, tr = sp2.sp2_density(h, wl.nocc)
        for n in range(1, tr.m + 2):
            t, q, e = tr.traces[n - 1], tr.sqnorms[n - 1], tr.errors[n - 1]
            e1 = tr.errors[n - 2] if n >= 2 else 0.0
            e2 = tr.errors[n - 3] if n >= 3 else 0.0
            e3 = tr.errors[n - 4] if n >= 4 else 0.0
            code = dm.sp2_decide(t, q, e, e1, e2, e3, n - 1, wl.n, wl.nocc, 10, 0.0)
            if n <= tr.m:
                assert code == tr.sigmas[n - 1], n
            else:
                assert code == 0


def test_controller_error_codes():
    import paper_2409_17033_amd as dm
    d = dm.sp2_decide     # (tr, sq, eps, eps_{n-1}, eps_{n-2}, eps_{n-3}, steps, n, nocc, ...)
    # bounds violations come first
    assert d(float("nan"), 1.0, 0.0, 0.0, 0.0, 0.0, 0, 10, 5) == -3
    assert d(5.0, 12.0, 0.0, 0.0, 0.0, 0.0, 0, 10, 5) == -3        # ||X||^2 > n + 1
    assert d(-2.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0, 10, 5) == -3
    assert d(5.0, float("inf"), 0.0, 0.0, 0.0, 0.0, 20, 10, 5) == -3
    # a state at x = 1/2 ((x - x^2)^2 = 1/16 >= 1/64) never stops, even stalled
    assert d(5.0, 4.75, 1 / 16, 1 / 16, 1 / 16, 1 / 16, 20, 10, 5) in (1, -1)
    # floor reached: eps stopped falling over two steps and is within 128 n u^2
    # (u = 2^-24; 128 * 10 * 2^-48 = 4.5e-12)
    assert d(5.0, 5.0, 1e-12, 1e-9, 1e-12, 1e-6, 20, 10, 5) == 0
    assert d(5.0, 5.0, 2e-12, 1e-9, 1e-12, 1e-6, 20, 10, 5) == 0
    # still falling: continue
    assert d(5.0, 5.0, 1e-12, 1e-6, 1e-9, 1e-3, 20, 10, 5) in (1, -1)
    # a single rise far above the floor does not stop (the previous test fell) ...
    assert d(5.0, 5.0, 1.2e-8, 3.1e-9, 3.5e-9, 1.4e-4, 20, 10, 5) in (1, -1)
    # ... a second rise in a row does, at any level below 1/64
    assert d(5.0, 5.0, 1.2e-8, 3.1e-9, 3.5e-9, 3.0e-9, 20, 10, 5) == 0
    assert d(5.0, 5.0, 1e-3, 1e-4, 1e-4, 1e-5, 20, 10, 5) == 0
    # the floor scales with n: the same single rise stops for n = 10^6 (5.8e-7)
    assert d(5e5, 5e5, 1.2e-8, 3.1e-9, 3.5e-9, 1.4e-4, 20, 10 ** 6, 5e5) == 0
    # the floor follows the product precision: two BF16 terms keep 16 bits
    # (128 * 10 * 2^-32 = 3.0e-7), so a single rise at 1.2e-8 is at their floor
    assert d(5.0, 5.0, 1.2e-8, 3.1e-9, 3.5e-9, 1.4e-4, 20, 10, 5, precision="split_bf16") == 0
    assert d(5.0, 5.0, 1.2e-8, 3.1e-9, 3.5e-9, 1.4e-4, 20, 10, 5, precision="split_fp16") in (1, -1)
    # one BF16 term keeps 8 bits: 128 * 10 * 2^-16 = 2.0e-2 reaches past 1/64,
    # so there the 1/64 resolution test is the only bound on a single rise
    assert d(5.0, 5.0, 1e-2, 1e-3, 5e-3, 1e-1, 20, 10, 5, precision="bf16") == 0
    assert d(5.0, 5.0, 1e-2, 1e-3, 5e-3, 1e-1, 20, 10, 5, precision="split_bf16") in (1, -1)
    assert d(5.0, 5.0, 2e-2, 1e-3, 5e-3, 1e-1, 20, 10, 5, precision="bf16") in (1, -1)
    # before min_iter no stop even at the floor
    assert d(5.0, 5.0, 1e-12, 1e-12, 1e-12, 1e-12, 3, 10, 5) in (1, -1)
    # exactly idempotent / idem_tol
    assert d(5.0, 5.0, 0.0, 0.0, 0.0, 0.0, 10, 10, 5) == 0
    assert d(5.0, 5.0, 5e-7, 1e-9, 1e-9, 1e-9, 20, 10, 5, 10, 1e-6) == 0


def test_nonorth_sizes_and_validation(lib):
    o = _opts(lib, 1000, 500)
    base = lib.dmpt_workspace_bytes(C.byref(o), 2)
    w = lib.dmpt_nonorth_workspace_bytes(C.byref(o), 2)
    # four padded n_pad^2 FP32 matrices and (2 + 2 nobs) n^2 FP32 matrices on top
    assert w >= base + 4 * 1024 * 1024 * 4 + 6 * 1000 * 1000 * 4
    assert lib.dmpt_nonorth_workspace_bytes(C.byref(o), 0) == 0
    out = (C.c_double * 1)()
    # NULL inputs are rejected before any device call
    assert lib.dmpt_susceptibility_nonorth(None, None, None, 1, None, None, None, out, C.byref(o), None) == 1
    assert lib.dmpt_susceptibility_nonorth(None, None, None, 0, None, None, None, out, C.byref(o), None) == 1


def test_fermi_validation(lib):
    from paper_2409_17033_amd._lib import FermiOpts
    o = _opts(lib, 1000, 500)
    f = FermiOpts(kt=0.01, mu=float("nan"), canonical=1)
    w = lib.dmpt_fermi_workspace_bytes(C.byref(o), C.byref(f), 2)
    assert w >= (6 + 2 + 4) * 1024 * 1024 * 4          # E, E^2, R, T, V, E_next, 2 Y, 4 temporaries
    for bad in (FermiOpts(kt=0.0, canonical=1), FermiOpts(kt=0.01, canonical=2),
                FermiOpts(kt=0.01, canonical=0, mu=float("nan")), FermiOpts(kt=0.01, canonical=1, doublings=41),
                FermiOpts(kt=0.01, canonical=1, reserved=1), FermiOpts(kt=0.01, canonical=1, count_tol=-1.0)):
        assert lib.dmpt_fermi_workspace_bytes(C.byref(o), C.byref(bad), 1) == 0
    # product formats: FP32, the FP16 split, the two- and three-term BF16 splits
    # (operand copies of 4, 4 and 6 bytes per element); plain BF16 and the
    # three-term-X^2 option are not offered here
    n_pad = 1024
    copies = 7 + 2                                      # E, E^2, R, T, E_next, S, W + 2 Y
    for prec, nbytes in ((5, 4), (1, 4), (2, 6)):
        sp = _opts(lib, 1000, 500, precision=prec)
        ws = lib.dmpt_fermi_workspace_bytes(C.byref(sp), C.byref(f), 2)
        assert ws - w == copies * nbytes * n_pad * n_pad, prec
    split = _opts(lib, 1000, 500, precision=3)
    assert lib.dmpt_fermi_workspace_bytes(C.byref(split), C.byref(f), 1) == 0
    split = _opts(lib, 1000, 500, precision=4)
    assert lib.dmpt_fermi_workspace_bytes(C.byref(split), C.byref(f), 1) == 0
    edge = _opts(lib, 1000, 0)                          # canonical needs 0 < nocc < n
    assert lib.dmpt_fermi_workspace_bytes(C.byref(edge), C.byref(f), 1) == 0
    out = (C.c_double * 1)()
    assert lib.dmpt_susceptibility_fermi(None, None, 1, None, None, out, C.byref(f), C.byref(o), None) == 1
    assert lib.dmpt_susceptibility_fermi(None, None, 1, None, None, out, C.byref(f), C.byref(split), None) == 7
