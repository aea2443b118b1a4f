"""Host-side checks of bench.py's contract (no GPU): more than one GPU is
refused with a message, and the committed HBM-traffic figure is used only
while the kernel sources and the job-list builder hash to the value recorded
with it."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_message():
    for extra in ([], ["--extra", "shapes"], ["--extra", "fermi"], ["--extra", "nonorth"]):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", *extra],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2
        assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_figure_follows_the_kernel_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    committed = bench.measured_traffic("split3x_bf16", 8192)
    assert committed is None or committed > 0
    # a copy of the tree whose kernel source differs: the figure is not used
    (tmp_path / "profiles").mkdir()
    src = os.path.join(ROOT, "profiles", "k_step_split3x_bf16_n8192_traffic.md")
    if os.path.exists(src):
        (tmp_path / "profiles" / "k_step_split3x_bf16_n8192_traffic.md").write_text(open(src).read())
    csrc = tmp_path / "paper_2409_17033_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "dmpt_kernels.hip").write_text("// changed\n")
    (csrc / "dmpt_internal.h").write_text("// changed\n")
    (csrc / "dmpt_lists.h").write_text("// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("split3x_bf16", 8192) is None
    assert bench.measured_traffic("no_such_precision", 8192) is None


def test_water_shaped_workload():
    """The Sec. VI water-cluster stand-in: 24 basis functions and 5 occupied
    orbitals per molecule, the gap opened to 2 % of the unshifted spectral
    width, one potential shift per atom (8 basis functions)."""
    import numpy as np

    import workloads as W
    wl = W.water_shaped(6, cache=False)
    assert (wl.n, wl.nocc) == (144, 30)
    h = wl.H.astype(np.float64)
    assert np.array_equal(wl.H, wl.H.T)
    w = np.linalg.eigvalsh(h)
    gap = w[wl.nocc] - w[wl.nocc - 1]
    # the shift moves only the virtual eigenvalues up by delta = gap -
    # gap_before, 0 < delta <= gap, and makes gap = 0.02 * (width - delta):
    # so 0.02 * (width - gap) <= gap <= 0.02 * width (a natural gap of a
    # random H at this size is far below 2 % of its width, so the shift applies)
    width = w[-1] - w[0]
    assert 0.02 * (width - gap) - 1e-6 <= gap <= 0.02 * width + 1e-6
    d = np.diag(wl.H1[0])
    assert np.count_nonzero(wl.H1[0] - np.diag(d)) == 0
    blocks = d.reshape(-1, 8)
    assert (blocks == blocks[:, :1]).all() and len(np.unique(blocks[:, 0])) == 18
    assert np.abs(d).max() <= 1.0
    assert np.array_equal(np.diag(wl.A[0]), np.arange(144, dtype=np.float32) - 71.5)


def test_path_names():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.path_kw("fp32") == dict(precision="fp32", refine=False, sweep_tol=0.0)
    assert bench.path_kw("split3x_bf16+refine") == dict(precision="split3x_bf16", refine=True, sweep_tol=0.0)
    assert bench.path_kw("split3x_bf16+refine@1e-3+project2") == dict(precision="split3x_bf16", refine=True,
                                                                      sweep_tol=1e-3, project=2)
    import pytest
    with pytest.raises(ValueError):
        bench.path_kw("split3x_bf16+refin")
