"""The ridge-round construction that mknn_build_device runs on the GPU, executed on the host
(tests/native/ridge_rounds_check.cpp): generated from pairs of tetrahedra sharing a
triangle, with no global order, its list entries must equal the sequential incremental
construction's exactly (Sec. 3: the lists depend only on the point sequence) -- on random
clouds, on an integer lattice (exact cospherical and coplanar sets everywhere) and on a flat
grid whose hull facets lie in one plane."""
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
    out = str(tmp_path_factory.mktemp("ridge") / "ridge_rounds_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC,
                    os.path.join(HERE, "native", "ridge_rounds_check.cpp"),
                    os.path.join(CSRC, "delaunay.cpp"), "-o", out], check=True)
    return out


@pytest.mark.parametrize("n,kind,seed", [(5, 0, 1), (60, 0, 2), (3000, 0, 3), (10_000, 0, 4),
                                         (1000, 1, 5), (2197, 1, 6), (904, 2, 7), (2504, 2, 8)])
def test_ridge_rounds_equal_sequential_lists(checker, n, kind, seed):
    r = subprocess.run([checker, str(n), str(kind), str(seed)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok"), r.stdout
