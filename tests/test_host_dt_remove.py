"""Vertex removal in the host triangulation kept for insertion: after removing sites, the
triangulation must equal the one built from scratch over the remaining sites (same
tetrahedra, ghosts included), stay structurally valid, and keep empty circumspheres.  On
degenerate input (an integer grid: many cospherical and coplanar sets) a removal may be
refused -- the caller then triangulates again -- but every accepted one must be exact."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2605_02224_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("dt") / "dt_remove_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(HERE, "native", "dt_remove_check.cpp"),
                    os.path.join(CSRC, "delaunay.cpp"), "-o", out], check=True)
    return out


@pytest.mark.parametrize("n,removals,seed,shape", [
    (200, 100, 1, 0), (2000, 1000, 4, 0), (3000, 2990, 9, 0),   # uniform cube, down to 10
    (300, 250, 2, 1), (400, 390, 7, 1),                          # sphere shell: all on the hull
])
def test_removal_equals_rebuild(checker, n, removals, seed, shape):
    r = subprocess.run([checker, str(n), str(removals), str(seed), str(shape)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")


@pytest.mark.parametrize("seed", [3, 11])
def test_removal_on_degenerate_grid_is_exact_or_refused(checker, seed):
    r = subprocess.run([checker, "300", "150", str(seed), "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode in (0, 3), r.stdout + r.stderr
    assert r.stdout.startswith("ok")
