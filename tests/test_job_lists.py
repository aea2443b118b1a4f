"""Host-side check of the step kernel's job lists (no GPU): the list builder
(paper_2409_17033_amd/csrc/dmpt_lists.h, the code the runtime uses) is
compiled into a small checker (tests/csrc/job_lists_check.cpp) and run over
the shapes below.  For each, every output tile of a step launch (each
observable's sweep tiles, and the X^2 tiles) must run exactly once: as a
regular job, inside a 256 x 256 wide job, or as the two K-split halves of
one scratch slot; no tile outside the upper triangle may appear; and the
lists must fit the workspace and split scratch the runtime reserves."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_17033_amd", "csrc")

# n_pad:nobs:with_p[:cus]; with_p = 1 is a step launch, 0 a sweep-only one
SHAPES = ["256:1:1", "512:1:1", "768:2:1", "1024:1:1", "1024:1:0", "1280:3:1", "2048:8:1", "2048:8:0",
          "4096:3:1", "7424:1:1", "7424:1:0", "8192:1:1", "8192:1:0", "8192:8:1", "8192:32:0",
          "16384:1:1", "16384:32:1", "8192:1:1:64", "8192:2:1:128", "4096:1:1:255", "2048:1:1:8"]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and not shutil.which(hipcc):
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("lists") / "job_lists_check")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", CSRC,
                        os.path.join(ROOT, "tests", "csrc", "job_lists_check.cpp"), "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def test_every_tile_runs_once(checker):
    r = subprocess.run([checker, *SHAPES], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("n_pad=")]
    assert len(lines) == len(SHAPES)
    # the headline shape uses both wide tiles and a K-split tail
    head = next(ln for ln in lines if ln.startswith("n_pad=8192 nobs=1 with_p=1 cus=256"))
    assert " 0 wide" not in head and " 0 split" not in head


def test_checker_sees_a_missing_tile(checker, tmp_path):
    """The checker itself: a copy of the list builder with one job dropped
    from every list must be reported."""
    src = open(os.path.join(CSRC, "dmpt_lists.h")).read()
    mark = "  append_xcd_ordered(L.jobs, rg);\n"
    assert mark in src
    (tmp_path / "dmpt_lists.h").write_text(src.replace(mark, mark + "  if (!L.jobs.empty()) L.jobs.erase(L.jobs.begin());\n"))
    hipcc = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = str(tmp_path / "bad_check")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-I", str(tmp_path), "-I", CSRC,
                        os.path.join(ROOT, "tests", "csrc", "job_lists_check.cpp"), "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe, "2048:1:1"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "FAIL" in r.stdout
