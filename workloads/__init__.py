"""Seeded synthetic inputs for the density-matrix susceptibility path.

This module is shared by the FP64 oracle tests and the GPU tests/benchmark. It
only *builds inputs* (Hamiltonians, observables, perturbations); it contains
none of the method's arithmetic (no SP2 step, no susceptibility formula).

The paper (Sec. VI) benchmarks on Hartree-Fock Fockians of water clusters that
are not available here; every workload below is a synthetic stand-in with the
shapes and spectral structure the method needs: a real symmetric H with a gap
at N_occ, symmetric observables, symmetric perturbations.

Recipes (seed = numpy ``default_rng([17033, cfg, n])``):

* ``dense_gapped``   (config 1, N=128): onsite ~ U(-1,1), off-diagonal
  ~ N(0, 0.1^2), then the virtual eigen-subspace is shifted up until the
  HOMO-LUMO gap at N_occ is >= 0.2.  A = (G+G^T)/2 with G ~ N(0,1).
* ``banded_gapped``  (config 2, N=4096; the N=8192 timed case uses the same
  recipe): half-bandwidth 64 (H_ij != 0 iff |i-j| <= 64), hopping
  ~ N(0, 0.05^2), onsite ~ U(-1,1), gap 0.1 opened the same way.
  A = diag(i - (N-1)/2), the centred site-position operator.
* perturbations H1: (G+G^T)/2, G ~ N(0,1), Frobenius-normalised.
* ``water_shaped``   (the matrix shapes of Sec. VI's water clusters, N = 24
  per molecule, N_occ = 5 per molecule): the config-2 recipe with the gap
  opened to 2 % of the spectral width, A = site position, H1 = a random
  potential shift per atom (8 basis functions each).

The gap is opened by H <- H + delta * (I - V_occ V_occ^T) where V_occ are the
N_occ lowest eigenvectors and delta = max(0, gap - (lambda_{occ+1} - lambda_occ)).
This keeps the eigenvectors and only moves the virtual eigenvalues, so the
gap is guaranteed (it also makes a banded H dense).

All matrices are returned as float32 (the precision the device path
consumes); tests promote the same float32 values to float64 for the oracle so
both sides see bit-identical inputs.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 17033


def rng_for(cfg: int, n: int, salt: int = 0) -> np.random.Generator:
    """Deterministic generator for workload ``cfg`` at size ``n``."""
    return np.random.default_rng([SEED_ROOT, cfg, n, salt])


def random_symmetric(rng: np.random.Generator, n: int, std: float = 1.0) -> np.ndarray:
    g = rng.normal(0.0, std, size=(n, n))
    return 0.5 * (g + g.T)


def frobenius_normalised(m: np.ndarray) -> np.ndarray:
    return m / np.linalg.norm(m)


def open_gap(h: np.ndarray, nocc: int, gap: float, relative: bool = False) -> np.ndarray:
    """Shift the virtual eigen-subspace of ``h`` so the gap at ``nocc`` is >= gap
    (>= gap times the spectral width of ``h`` when ``relative``).

    For n >= 2048 the eigenvectors come from an FP32 divide-and-conquer
    eigensolver (scipy 'evd'): the shift only needs the occupied subspace to
    ~1e-6, which moves the opened gap by the same amount.
    """
    n = h.shape[0]
    if nocc <= 0 or nocc >= n:
        return h
    if n >= 2048:
        import scipy.linalg as sl
        w, v = sl.eigh(h.astype(np.float32), driver="evd")
        w, v = w.astype(np.float64), v.astype(np.float64)
    else:
        w, v = np.linalg.eigh(h)
    if relative:
        gap = gap * (w[-1] - w[0])
    delta = max(0.0, gap - (w[nocc] - w[nocc - 1]))
    if delta == 0.0:
        return h
    vv = v[:, nocc:]
    out = h + delta * (vv @ vv.T)
    return 0.5 * (out + out.T)


def banded_mask(n: int, half_bandwidth: int) -> np.ndarray:
    i = np.arange(n)
    return np.abs(i[:, None] - i[None, :]) <= half_bandwidth


def position_observable(n: int) -> np.ndarray:
    """Centred site-position operator diag(i - (n-1)/2)."""
    return np.diag(np.arange(n, dtype=np.float64) - 0.5 * (n - 1))


@dataclass
class Workload:
    name: str
    n: int
    nocc: int
    H: np.ndarray                      # float32 (n, n)
    A: np.ndarray                      # float32 (nobs, n, n)
    H1: np.ndarray                     # float32 (npert, n, n)
    meta: dict = field(default_factory=dict)


def _as32(m: np.ndarray) -> np.ndarray:
    m32 = np.ascontiguousarray(m, dtype=np.float32)
    # Exact symmetry of the float32 copy (rounding a symmetric FP64 matrix
    # is already symmetric, this only guards against asymmetric round-off in
    # the generators themselves).
    if m32.ndim == 2:
        m32 = np.triu(m32) + np.triu(m32, 1).T
    return m32


def dense_gapped(n: int = 128, nocc: int | None = None, gap: float = 0.2,
                 npert: int = 8, nobs: int = 1, cfg: int = 1) -> Workload:
    """Config 1: dense random symmetric H with a gap at nocc."""
    nocc = n // 2 if nocc is None else nocc
    rng = rng_for(cfg, n)
    off = rng.normal(0.0, 0.1, size=(n, n))
    h = np.triu(off, 1)
    h = h + h.T
    h[np.diag_indices(n)] = rng.uniform(-1.0, 1.0, size=n)
    h = open_gap(h, nocc, gap)
    a = np.stack([random_symmetric(rng, n) for _ in range(nobs)])
    h1 = np.stack([frobenius_normalised(random_symmetric(rng, n)) for _ in range(npert)])
    return Workload("dense_gapped", n, nocc, _as32(h),
                    np.stack([_as32(x) for x in a]), np.stack([_as32(x) for x in h1]),
                    {"gap": gap, "cfg": cfg})


def banded_gapped(n: int = 4096, nocc: int | None = None, gap: float = 0.1,
                  half_bandwidth: int = 64, hop_std: float = 0.05, npert: int = 8,
                  observable: str = "position", nobs: int = 1, cfg: int = 2,
                  cache: bool = True) -> Workload:
    """Config 2 (and the N=8192 timed case): banded tight-binding H with a gap."""
    nocc = n // 2 if nocc is None else nocc
    key = f"banded_c{cfg}_n{n}_o{nocc}_g{gap}_b{half_bandwidth}_{observable}_{nobs}_{npert}"
    cdir = os.environ.get("DMPT_WORKLOAD_CACHE")
    path = os.path.join(cdir, key + ".npz") if (cache and cdir) else None
    if path and os.path.exists(path):
        z = np.load(path)
        return Workload("banded_gapped", n, nocc, z["H"], z["A"], z["H1"],
                        {"gap": gap, "cfg": cfg, "half_bandwidth": half_bandwidth})
    rng = rng_for(cfg, n)
    hop = rng.normal(0.0, hop_std, size=(n, n))
    hop = np.triu(hop, 1) * banded_mask(n, half_bandwidth)
    h = hop + hop.T
    h[np.diag_indices(n)] = rng.uniform(-1.0, 1.0, size=n)
    h = open_gap(h, nocc, gap)
    if observable == "position":
        a = np.stack([position_observable(n)] * nobs)
    else:
        a = np.stack([frobenius_normalised(random_symmetric(rng, n)) for _ in range(nobs)])
    h1 = np.stack([frobenius_normalised(random_symmetric(rng, n)) for _ in range(npert)])
    wl = Workload("banded_gapped", n, nocc, _as32(h),
                  np.stack([_as32(x) for x in a]), np.stack([_as32(x) for x in h1]),
                  {"gap": gap, "cfg": cfg, "half_bandwidth": half_bandwidth})
    if path:
        try:                       # the cache is an optimisation only
            os.makedirs(cdir, exist_ok=True)
            np.savez(path + ".tmp.npz", H=wl.H, A=wl.A, H1=wl.H1)
            os.replace(path + ".tmp.npz", path)
        except OSError:
            pass
    return wl


def banded_gapless(n: int = 16384, nocc: int | None = None, half_bandwidth: int = 256, hop_std: float = 0.05,
                   nobs: int = 32, cfg: int = 5, log=None) -> Workload:
    """Config 5 (finite temperature): random banded H (half-bandwidth 256,
    hopping ~ N(0, hop_std^2), onsite ~ U(-1, 1)) with no gap opened, and
    nobs random symmetric Frobenius-normalised observables.  log: optional
    callable told about each observable as it is drawn (large batches take
    minutes)."""
    nocc = n // 2 if nocc is None else nocc
    rng = rng_for(cfg, n)
    hop = rng.normal(0.0, hop_std, size=(n, n))
    hop = np.triu(hop, 1) * banded_mask(n, half_bandwidth)
    h = hop + hop.T
    h[np.diag_indices(n)] = rng.uniform(-1.0, 1.0, size=n)
    a = np.zeros((nobs, n, n), np.float32)
    for k in range(nobs):
        a[k] = _as32(frobenius_normalised(random_symmetric(rng, n)))
        if log:
            log(f"observable {k + 1} of {nobs} drawn")
    return Workload("banded_gapless", n, nocc, _as32(h), a, np.zeros((0, n, n), np.float32),
                    {"cfg": cfg, "half_bandwidth": half_bandwidth})


def water_shaped(molecules: int, cfg: int = 6, gap_rel: float = 0.02,
                 basis_per_atom: int = 8, cache: bool = True) -> Workload:
    """Stand-in with the shapes of the water-cluster test of Sec. VI (Table 2:
    100, 190 and 301 molecules give N = 2400, 4560, 7224).

    N = 3 atoms x 8 basis functions per molecule, N_occ = 5 doubly occupied
    orbitals per molecule (10 electrons, restricted).  H follows the config-2
    recipe (half-bandwidth 64, hopping ~ N(0, 0.05^2), onsite ~ U(-1, 1)) with
    the gap at N_occ opened to ``gap_rel`` of the spectral width before the
    shift (the paper prints no spectra; 2 % is an assumption).  A = centred site position
    (stand-in for the x dipole operator).  One perturbation H1: a random
    potential shift ~ U(-1, 1) on each atom, i.e. diagonal and constant over
    the atom's block of basis functions.
    """
    n = 3 * basis_per_atom * molecules
    nocc = 5 * molecules
    key = f"water_c{cfg}_m{molecules}_g{gap_rel}_b{basis_per_atom}"
    cdir = os.environ.get("DMPT_WORKLOAD_CACHE")
    path = os.path.join(cdir, key + ".npz") if (cache and cdir) else None
    meta = {"cfg": cfg, "molecules": molecules, "gap_rel": gap_rel, "half_bandwidth": 64}
    if path and os.path.exists(path):
        z = np.load(path)
        return Workload("water_shaped", n, nocc, z["H"], z["A"], z["H1"], meta)
    rng = rng_for(cfg, n)
    hop = rng.normal(0.0, 0.05, size=(n, n))
    hop = np.triu(hop, 1) * banded_mask(n, 64)
    h = hop + hop.T
    h[np.diag_indices(n)] = rng.uniform(-1.0, 1.0, size=n)
    h = open_gap(h, nocc, gap_rel, relative=True)
    shifts = np.repeat(rng.uniform(-1.0, 1.0, size=3 * molecules), basis_per_atom)
    wl = Workload("water_shaped", n, nocc, _as32(h), _as32(position_observable(n))[None],
                  _as32(np.diag(shifts))[None], meta)
    if path:
        try:                       # the cache is an optimisation only
            os.makedirs(cdir, exist_ok=True)
            np.savez(path + ".tmp.npz", H=wl.H, A=wl.A, H1=wl.H1)
            os.replace(path + ".tmp.npz", path)
        except OSError:
            pass
    return wl


def scf_system(n: int = 1024, cfg: int = 4, ntrain: int = 40):
    """Self-consistent response case (config 4): banded gapped H0 (the config-2
    recipe at size n), on-site interactions U_i ~ U(0.5, 1.5), the test
    observable A = site position, an external field H1 = diag(N(0, 0.01^2)),
    and `ntrain` random symmetric Frobenius-normalised observables whose
    linear-mixing runs provide the mixer's training pairs.
    Returns (workload, U (float32), training observables (float32))."""
    wl = banded_gapped(n, cfg=cfg, npert=1, cache=False)
    rng = rng_for(cfg, n, 1)
    u = rng.uniform(0.5, 1.5, size=n).astype(np.float32)
    h1 = np.diag(rng.normal(0.0, 0.01, size=n))[None]
    train = np.stack([_as32(frobenius_normalised(random_symmetric(rng, n))) for _ in range(ntrain)]) \
        if ntrain else np.zeros((0, n, n), np.float32)
    wl = Workload("scf_system", n, wl.nocc, wl.H, wl.A, np.stack([_as32(x) for x in h1]),
                  {"cfg": cfg, "half_bandwidth": 64})
    return wl, u, train


def known_spectrum(n: int, nocc: int, gap: float = 0.3, seed: int = 0,
                   width: float = 2.0) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """H = Q diag(w) Q^T with a chosen ascending spectrum and a random orthogonal Q.

    Returns (H, w, Q) in float64; the exact eigenpairs are known by construction.
    """
    rng = rng_for(99, n, seed)
    q, r = np.linalg.qr(rng.normal(size=(n, n)))
    q = q * np.sign(np.diag(r))
    lo = np.sort(rng.uniform(-width / 2, -gap / 2, size=nocc))
    hi = np.sort(rng.uniform(gap / 2, width / 2, size=n - nocc))
    w = np.concatenate([lo, hi])
    h = (q * w) @ q.T
    return 0.5 * (h + h.T), w, q


def gapless(n: int, nocc: int, seed: int = 0) -> np.ndarray:
    """Symmetric H whose HOMO and LUMO are exactly degenerate (no gap at nocc)."""
    rng = rng_for(98, n, seed)
    q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    w = np.sort(rng.uniform(-1, 1, size=n))
    w[nocc] = w[nocc - 1]
    h = (q * w) @ q.T
    return 0.5 * (h + h.T)


def random_perturbations(n: int, count: int, seed: int = 0) -> np.ndarray:
    rng = rng_for(97, n, seed)
    return np.stack([frobenius_normalised(random_symmetric(rng, n)) for _ in range(count)])
