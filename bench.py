"""Time-to-chi benchmark on one MI355X.

One "step" is one pass of the whole hot path for one synthetic problem:
spectral bounds -> X_1, Y_1 -> SP2 recursion merged with the susceptibility
sweep (Eq. DMSuscept) with device-side sigma/stop decisions -> occupied-virtual
projection -> (with "+refine": the residual correction of chi) -> D, chi, a0
-> responses Tr[chi H1] for 8 perturbations (Eq. dual).

A path is a product precision, optionally with "+refine", and then with
"@t": the sweeps stop once X_n is within t of idempotency (sweep_tol), the
correction's within sqrt(t); the correction removes what that leaves.  The
headline is a BF16 path (the metric is split-BF16 against FP32); every path's
D, chi and a0 are compared once, outside the timed region, with the FP64
closed form (one eigendecomposition on the host), and reported with its time.

Workload: N = 8192, N_occ = 4096, banded tight-binding H (half-bandwidth 64,
hopping ~ N(0, 0.05^2), onsite ~ U(-1, 1)) with a 0.1 gap opened at N_occ,
A = centred site-position operator, 8 Frobenius-normalised random H1
(synthetic stand-in for the paper's water-cluster Fockians, which are not
available).  Inputs are resident in HBM before the timed region.

Prints one JSON line.  --gpus N with N > 1 exits: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-χ (ms) + MFMA TFLOP/s at N=8192, split-BF16 vs FP32, at stated error"
PEAK = {"bf16": 2516.6, "f16": 2516.6, "fp32": 157.3}          # dense MFMA TFLOP/s (MI355X)
# MFMA products per FP32-equivalent product: (X^2, YX + XY) of one step
PRODUCTS = {"split3_bf16": (6, 6), "split3x_bf16": (6, 3), "split_bf16": (3, 3), "split_fp16": (3, 3),
            "fp32": (1, 1), "bf16": (1, 1)}


def step_flops(prec, n_pad, m, sweep_steps, nobs=1):
    """Executed MFMA flops of the m step launches on the upper-triangle
    tiles: X^2 as a symmetric rank-n product (n^3 per product) in every
    launch, YX + XY (2 n^3 per product) in the first sweep_steps launches
    (all of them unless the sweep stopped early)."""
    px, pz = PRODUCTS[prec]
    n3 = float(n_pad) ** 3
    return n3 * (m * px + sweep_steps * nobs * 2 * pz)


# The dominant kernel of each path: the step launch (for split3x one mixed
# launch: X^2 tiles in the three-term split, sweep tiles in the two-term one).
KERNEL = {"split3x_bf16": "k_step<split3_bf16 X^2, split_bf16 sweep> (one mixed launch per SP2 + chi step)"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--precision", default="split3x_bf16+refine@1e-3",
                    help="headline path: a precision, optionally with +refine (the residual correction) "
                         "and @t (the sweeps stop at sweep_tol t), and +project2 (the projections above "
                         "the sweep's precision)")
    ap.add_argument("--compare", default="fp32,split3_bf16,split_fp16,split3x_bf16+refine,"
                                         "split3x_bf16+refine@1e-3+project2,split_fp16+refine,split_bf16",
                    help="other paths timed for context")
    ap.add_argument("--compare-steps", type=int, default=1)
    ap.add_argument("--no-errors", action="store_true", help="skip the closed-form errors of each path")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=5, help="FP64 oracle SP2+chi steps in the CPU sample")
    ap.add_argument("--cpu-full", action="store_true",
                    help="CPU baseline in full instead of the bounded sample: the whole FP64 recursion and "
                         "the closed form on all host threads, and one recursion step and the closed form "
                         "of the same recipe at N/2 on one thread")
    ap.add_argument("--nobs", type=int, default=1, help="--extra fermi: observables in one batch")
    ap.add_argument("--no-fp32", action="store_true", help="--extra fermi|nonorth: time args.precision only")
    ap.add_argument("--extra", choices=["fermi", "nonorth", "shapes"], default=None,
                    help="instead of the headline metric, time the finite-temperature path (Sec. V.B: "
                         "gapless banded H, kT = 0.01, one random observable), the non-orthonormal one "
                         "(Sec. V.A: the headline workload with Z = I + 1e-3 G), or the water-cluster "
                         "shapes of Sec. VI (N = 2400, 4560, 7224; both duality routes) and print their "
                         "own JSON line")
    return ap.parse_args()


def run_shapes(args, dm, torch, W, dev):
    """The matrix shapes of Sec. VI's water clusters (Table 2): for 100, 190 and
    301 molecules, time-to-chi and the step kernel's rate in args.precision,
    the FP16 split (the analogue of the paper's FP16 tensor-core runs) and
    FP32, and the first-order response by both routes of the duality:
    Tr[chi^A H1] (timed) and s Tr[A D1] (D1 from the same recursion with H1 in
    place of A).  Prints one JSON line."""
    shapes = []
    for mol in (100, 190, 301):
        t = time.perf_counter()
        wl = W.water_shaped(mol)
        log(f"water-shaped N={wl.n} generated in {time.perf_counter() - t:.1f} s")
        H, A, H1 = (torch.from_numpy(x).to(dev) for x in (wl.H, wl.A[0], wl.H1[0]))
        n_pad = -(-wl.n // 256) * 256
        row = {"molecules": mol, "n": wl.n, "nocc": wl.nocc, "n_pad": n_pad, "paths": {}}
        for path in dict.fromkeys([args.precision, "split_fp16", "fp32"]):
            prec = path.partition("+")[0]
            ms, chi, D, a0, resp, infos = run_path(dm, torch, H, A, H1, wl.nocc, path, args.steps, args.warmup)
            info = infos[-1]
            m = info["m"]
            step_avg = info["step_ms"] / max(m, 1)
            executed = step_flops(prec, n_pad, m, info["sweep_steps"]) / (info["step_ms"] * 1e-3) / 1e12
            d1, _, _, info1 = dm.susceptibility(H, H1, wl.nocc, spin=1.0, want_density=False, **path_kw(path))
            r_d1 = 2.0 * float(dm.response(d1, A)[0, 0])
            row["paths"][path] = {
                "ms": round(ms, 3), "m": m, "step_avg_ms": round(step_avg, 4),
                "mfma_tflops": round(executed, 1), "mfma_tflops_fma1": round(executed / 2, 1),
                "algorithmic_tflops": round(3.0 * float(wl.n) ** 3 * m / (ms * 1e-3) / 1e12, 1),
                "tr_chi_h1": float(resp[0, 0]), "s_tr_a_d1": r_d1, "m_d1": info1["m"],
                "props": property_errors(torch, H, A, D, chi, wl.nocc, 2.0),
            }
            log(f"N={wl.n} {path}: {ms:.1f} ms  M={m}  step {step_avg:.3f} ms  MFMA {executed:.1f} TF/s  "
                f"Tr[chi H1]={resp[0, 0]:.8f}  2Tr[A D1]={r_d1:.8f}")
            del chi, D, d1
            torch.cuda.empty_cache()
        shapes.append(row)
        del H, A, H1
    print(json.dumps({"extra": "shapes", "unit": "ms", "steps": args.steps, "warmup": args.warmup,
                      "data": "synthetic",
                      "config": {"workload": "water-cluster shapes of Sec. VI: N = 24 and N_occ = 5 per "
                                             "molecule, config-2 banded H with the gap at 2 % of the width, "
                                             "A = site position, H1 = one potential shift per atom"},
                      "shapes": shapes}), flush=True)


def run_extra(args, dm, torch, W, dev):
    """Time one of the Sec. V paths in args.precision and FP32 (steps timed
    calls after warmup ones, inputs resident); prints one JSON line."""
    t = time.perf_counter()
    if args.extra == "fermi":
        wl = W.banded_gapless(args.n, half_bandwidth=256, nobs=args.nobs, log=log)
        H, A = torch.from_numpy(wl.H).to(dev), torch.from_numpy(wl.A).to(dev)
        call = lambda prec: dm.susceptibility_fermi(H, A, wl.nocc, 0.01, precision=prec)
        workload = (f"gapless banded H (half-bandwidth 256), N={wl.n}, N_occ={wl.nocc}, kT=0.01, "
                    f"{args.nobs} random observable(s) in one batch")
    else:
        wl = W.banded_gapped(args.n, cfg=2)
        H, A = torch.from_numpy(wl.H).to(dev), torch.from_numpy(wl.A[0]).to(dev)
        g = torch.Generator(device=dev).manual_seed(0)
        Z = torch.eye(wl.n, device=dev) + 1e-3 * torch.randn(wl.n, wl.n, device=dev, generator=g)
        call = lambda prec: dm.susceptibility_nonorth(H, Z, A, wl.nocc, precision=prec)
        workload = f"headline workload N={wl.n} in a basis with inverse factor Z = I + 1e-3 G"
    log(f"{args.extra} workload N={wl.n} generated in {time.perf_counter() - t:.1f} s")
    torch.cuda.synchronize()
    paths = {}
    base = args.precision.partition("+")[0]
    if args.extra == "fermi" and base == "split3x_bf16":
        base = "split3_bf16"   # the finite-temperature products take one format for all operands
    for prec in dict.fromkeys([base] if args.no_fp32 else [base, "fp32"]):
        for _ in range(args.warmup):
            call(prec)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            out = call(prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / max(args.steps, 1)
        info = out[-1]
        paths[prec] = {"ms": round(ms, 3), "device_ms": round(info["elapsed_ms"], 3)}
        if args.extra == "fermi":
            paths[prec].update({"mu": info["mu"], "doublings": info["doublings"], "newton": info["newton"],
                                "products": info["products"]})
        else:
            paths[prec]["m"] = info["m"]
        log(f"{args.extra} {prec}: {ms:.1f} ms  {paths[prec]}")
    print(json.dumps({"extra": args.extra, "unit": "ms", "steps": args.steps, "warmup": args.warmup,
                      "data": "synthetic", "config": {"workload": workload, "n": wl.n}, "paths": paths}), flush=True)


def property_errors(torch, H, A, D, chi, nocc, spin):
    """Checks that hold at any size: idempotency, trace, symmetry, Tr chi = 0 and
    the commutator identity [H, chi'] = [D, A] (chi' = chi / s), on the device
    in FP64 (cast copies)."""
    Hd, Ad, Dd, Cd = H.double(), A.double(), D.double(), chi.double() / spin
    out = {}
    out["idempotency"] = (torch.linalg.norm(Dd @ Dd - Dd) / torch.linalg.norm(Dd)).item()
    out["trace_d_minus_nocc"] = (torch.trace(Dd) - nocc).item()
    out["chi_asymmetry"] = torch.linalg.norm(Cd - Cd.T).item()
    out["trace_chi_rel"] = (torch.trace(Cd).abs() / (torch.linalg.norm(Cd) * Cd.shape[0] ** 0.5)).item()
    da = Dd @ Ad
    lhs = Hd @ Cd - Cd @ Hd
    rhs = da - da.T
    out["commutator_residual"] = (torch.linalg.norm(lhs - rhs) / torch.linalg.norm(rhs)).item()
    return out


def path_kw(path):
    """Options of a path "precision[+refine[@sweep_tol]][+project2]"."""
    parts = path.split("+")
    kw = dict(precision=parts[0], refine=False, sweep_tol=0.0)
    for part in parts[1:]:
        if part.startswith("refine"):
            tol = part.partition("@")[2]
            kw.update(refine=True, sweep_tol=float(tol) if tol else 0.0)
        elif part == "project2":
            kw["project"] = 2
        else:
            raise ValueError(f"unknown path option {part!r} in {path!r}")
    return kw


def run_path(dm, torch, H, A, H1, nocc, path, steps, warmup):
    kw = dict(path_kw(path), profile=True)
    for _ in range(warmup):
        chi, D, a0, info = dm.susceptibility(H, A, nocc, **kw)
        dm.response(chi, H1)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        chi, D, a0, info = dm.susceptibility(H, A, nocc, **kw)
        resp = dm.response(chi, H1)
        infos.append(info)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    return ms, chi, D, a0, resp, infos


def closed_form(wl):
    """FP64 closed form of the workload on the host (test infrastructure, off
    the timed region): D, chi = s L o A, a0 = s Tr[A D]; also its wall time."""
    import numpy as np
    from oracle import closed_form as cf
    t = time.perf_counter()
    h, a = wl.H.astype(np.float64), wl.A[0].astype(np.float64)
    w, v = cf.eigensystem(h)
    vo = v[:, :wl.nocc]
    d = vo @ vo.T
    chi = 2.0 * (v @ (cf.loewner_step(w, wl.nocc) * (v.T @ a @ v)) @ v.T)
    a0 = 2.0 * cf.expectation(a, d)
    return {"d": d, "chi": chi, "a0": a0, "seconds": time.perf_counter() - t}


def path_errors(ref, D, chi, a0, resp, wl):
    """Relative Frobenius errors of D and chi, the response error relative to
    ||chi_ref||_F (the H1 are Frobenius-normalised: Cauchy-Schwarz) and the
    a0 error relative to 2 ||A||_F ||D_ref||_F."""
    import numpy as np
    from oracle import closed_form as cf
    c = chi.double().cpu().numpy()
    rref = cf.response(ref["chi"], wl.H1)
    a64 = wl.A[0].astype(np.float64)
    return {"d": cf.rel_frobenius(D.double().cpu().numpy(), ref["d"]),
            "chi": cf.rel_frobenius(c, ref["chi"]),
            "response": float(np.max(np.abs(np.asarray(resp)[0] - rref)) / np.linalg.norm(ref["chi"])),
            "a0": abs(a0[0] - ref["a0"]) / (2.0 * np.linalg.norm(a64) * np.linalg.norm(ref["d"]))}


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max((p.get("num_threads", 0) for p in threadpool_info()), default=os.cpu_count())
    except Exception:
        return os.cpu_count()


def _oracle_steps(wl, steps):
    """Seconds per step of the FP64 oracle's merged recursion (Eq. DMSuscept)
    over `steps` steps (all of them when steps is None: the oracle's own
    stopping rule), and the steps run."""
    import numpy as np
    from oracle import sp2
    h = wl.H.astype(np.float64)
    a = wl.A[0].astype(np.float64)
    t0 = time.perf_counter()
    if steps is None:
        out = sp2.sp2_susceptibility(h, a, wl.nocc)
        m = out[-1].m if hasattr(out[-1], "m") else len(out[-1].sigmas)
        return (time.perf_counter() - t0) / max(m, 1), m
    emin, emax = sp2.gershgorin_bounds(h)
    alpha, beta = sp2.sp2_coefficients(emin, emax)
    x = alpha * np.eye(wl.n) + beta * h
    y = beta * a
    t0 = time.perf_counter()
    for _ in range(steps):
        s = sp2.choose_sigma(np.trace(x), np.sum(x * x), wl.nocc)
        y = sp2.response_update(y, x, s)
        x = sp2.sp2_update(x, s)
    return (time.perf_counter() - t0) / steps, steps


def cpu_baseline(wl, m_steps, steps, closed_s):
    """The FP64 oracle on the host cores: `steps` steps of its merged
    recursion (Eq. DMSuscept) at the full size, scaled to the GPU's step
    count M; the closed form's wall time (eigendecomposition + Loewner
    product) beside it."""
    per_step, _ = _oracle_steps(wl, steps)
    return {
        "value": per_step * m_steps * 1e3,
        "unit": "ms",
        "cores": _threads(),
        "kind": "oracle",
        "sample": f"{steps} FP64 SP2+chi step(s) (Eq. DMSuscept, numpy GEMMs) at N={wl.n}, "
                  f"{per_step:.2f} s/step, scaled to the GPU's M={m_steps} steps",
        "closed_form_ms": round(closed_s * 1e3, 1) if closed_s else None,
    }


def cpu_baseline_full(wl, W, closed_s):
    """The CPU baseline in full: the oracle's whole FP64 recursion (its own
    sigma and stopping rules) and the closed form on all host threads; on one
    thread (threadpoolctl) one recursion step and the closed form of the same
    recipe at N/2, each with its N^3 scaling to the full size."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import closed_form as cf
    out = {"cores": _threads()}
    t0 = time.perf_counter()
    per_step, m = _oracle_steps(wl, None)
    out["recursion_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    out["recursion_steps"] = m
    out["closed_form_ms"] = round(closed_s * 1e3, 1)
    half = W.banded_gapped(wl.n // 2, cfg=2)
    with threadpool_limits(limits=1):
        step1, _ = _oracle_steps(half, 1)
        t0 = time.perf_counter()
        h = half.H.astype(np.float64)
        w, v = cf.eigensystem(h)
        _ = v @ (cf.loewner_step(w, half.nocc) * (v.T @ half.A[0].astype(np.float64) @ v)) @ v.T
        cf1 = time.perf_counter() - t0
    out["one_thread"] = {"n": half.n, "recursion_step_ms": round(step1 * 1e3, 1),
                         "closed_form_ms": round(cf1 * 1e3, 1),
                         "recursion_ms_scaled_to_full_n": round(step1 * 8 * m * 1e3, 1),
                         "closed_form_ms_scaled_to_full_n": round(cf1 * 8 * 1e3, 1)}
    return out


def measured_traffic(prec, n):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a copy kernel), used only
    while the kernel sources and the job-list builder (which sets the order
    the tiles stream through L2) still hash to the value recorded with it."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_step_{prec}_n{n}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for src in ("paper_2409_17033_amd/csrc/dmpt_kernels.hip", "paper_2409_17033_amd/csrc/dmpt_internal.h",
                "paper_2409_17033_amd/csrc/dmpt_lists.h"):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if fields.get("kernel_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2409_17033_amd as dm
    import workloads as W

    dm.load()
    dev = torch.device("cuda:0")
    if args.extra == "shapes":
        run_shapes(args, dm, torch, W, dev)
        return
    if args.extra:
        run_extra(args, dm, torch, W, dev)
        return
    t = time.perf_counter()
    wl = W.banded_gapped(args.n, cfg=2)
    log(f"workload N={wl.n} generated in {time.perf_counter() - t:.1f} s")
    H = torch.from_numpy(wl.H).to(dev)
    A = torch.from_numpy(wl.A[0]).to(dev)
    H1 = torch.from_numpy(wl.H1).to(dev)
    torch.cuda.synchronize()

    ref = None
    if not args.no_errors:
        t = time.perf_counter()
        ref = closed_form(wl)
        log(f"closed form (FP64 eigendecomposition on {_threads()} host threads) in {time.perf_counter() - t:.1f} s")

    results = {}
    for path, steps, warm in [(args.precision, args.steps, args.warmup)] + \
            [(p, args.compare_steps, 1) for p in args.compare.split(",") if p and p != args.precision]:
        prec = path.partition("+")[0]
        ms, chi, D, a0, resp, infos = run_path(dm, torch, H, A, H1, wl.nocc, path, steps, warm)
        info = infos[-1]
        props = property_errors(torch, H, A, D, chi, wl.nocc, 2.0)
        m = info["m"]
        n_pad = -(-wl.n // 256) * 256
        flops = step_flops(prec, n_pad, m, info["sweep_steps"])   # executed MFMA flops of the m step launches
        step_avg_ms = info["step_ms"] / max(m, 1)
        results[path] = {
            "ms": ms, "m": m, "step_ms_total": info["step_ms"], "step_avg_ms": step_avg_ms,
            "bounds_ms": info["bounds_ms"], "project_ms": info["project_ms"], "refine_ms": info["refine_ms"],
            "output_ms": info["output_ms"], "elapsed_ms": info["elapsed_ms"],
            "sweep_steps": info["sweep_steps"], "correction_steps": info["correction_steps"],
            "mfma_tflops": flops / (info["step_ms"] * 1e-3) / 1e12 if info["step_ms"] > 0 else None,
            "algorithmic_tflops": 3.0 * float(wl.n) ** 3 * m / (ms * 1e-3) / 1e12,
            "a0": a0[0], "props": props,
            "errors": path_errors(ref, D, chi, a0, resp, wl) if ref is not None else None,
        }
        log(f"{path}: {ms:.1f} ms/step  M={m}  kernel avg {step_avg_ms:.2f} ms/step  "
            f"MFMA {results[path]['mfma_tflops']:.1f} TF/s  errors {results[path]['errors']}")
        del chi, D
        torch.cuda.empty_cache()

    main_path = args.precision
    main_prec = main_path.partition("+")[0]
    r = results[main_path]
    dtype = "fp32" if main_prec == "fp32" else "f16" if main_prec == "split_fp16" else "bf16"
    roof = {
        "bound": "mfma",
        "kernel": KERNEL.get(main_prec, f"k_step<{main_prec}> (one SP2 + chi step)"),
        "achieved": r["mfma_tflops"],
        "peak": PEAK[dtype],
        "unit": "TFLOP/s",
        "frac": r["mfma_tflops"] / PEAK[dtype] if r["mfma_tflops"] else None,
        "traffic": measured_traffic(main_prec, args.n),
    }
    cpu = None
    if not args.no_cpu:
        t = time.perf_counter()
        closed_s = ref["seconds"] if ref is not None else None
        if args.cpu_full:
            cpu = cpu_baseline(wl, r["m"], args.cpu_steps, closed_s)
            cpu["full"] = cpu_baseline_full(wl, W, closed_s)
        else:
            cpu = cpu_baseline(wl, r["m"], args.cpu_steps, closed_s)
        log(f"cpu baseline in {time.perf_counter() - t:.1f} s: {cpu}")
    fp32 = results.get("fp32")
    line = {
        "metric": METRIC,
        "value": round(r["ms"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": f"banded gapped tight-binding H, N={wl.n}, N_occ={wl.nocc}, half-bandwidth 64, "
                        "gap 0.1, A = site position, 8 random H1",
            "n": wl.n, "nocc": wl.nocc, "path": main_path,
            "sweep": "forward merged (Eq. DMSuscept) + occupied-virtual projection"
                     + (" + residual correction" if path_kw(main_path)["refine"] else "")
                     + (f", sweeps stopped at sweep_tol {path_kw(main_path)['sweep_tol']:g}"
                        if path_kw(main_path)["sweep_tol"] else ""),
            "bounds": "lanczos",
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "paths": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in results.items()},
        "speedup_vs_fp32": (fp32["ms"] / r["ms"]) if fp32 and main_path != "fp32" else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
