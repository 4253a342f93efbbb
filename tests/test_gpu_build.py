"""Successor lists built on the GPU (mknn_build_device) against the host construction
(mknn_build): the same lists, entry for entry (Sec. 3: the lists are a function of the
point sequence, not of how the construction is scheduled).  The host construction is
itself pinned against the oracle's exact lists (tests/test_host_build.py)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_02224_amd import api as A
    from paper_2605_02224_amd import workloads as W
    from paper_2605_02224_amd import _lib
    return torch, A, W, _lib


def _same_lists(A, pts, order=None):
    print(f"device build: n={pts.shape[0]}", flush=True)
    host = A.Cloud.build(pts, order)
    dev = A.Cloud.build(pts, order, device=True)
    st = A.build_device_stats()
    ho, he = host.successors()
    do, de = dev.successors()
    assert np.array_equal(ho, do), "list offsets differ"
    assert np.array_equal(he, de), "list entries differ"
    assert np.array_equal(host.points_by_rank(), dev.points_by_rank())
    return st, dev


@pytest.mark.parametrize("n,shape,seed", [(5, "sphere", 1), (64, "sphere", 2),
                                          (20_000, "sphere", 0), (50_000, "torus", 3),
                                          (100_000, "ellipsoid", 4)])
def test_device_lists_equal_host(env, n, shape, seed):
    torch, A, W, _ = env
    c = W.random_cloud(n, seed, shape)
    st, _ = _same_lists(A, c.points, c.order)
    if n >= 5 and st["rounds"]:
        assert st["entries"] == int(A.Cloud.build(c.points, c.order).successors()[0][-1])


def test_device_lists_lattice(env):
    """Integer lattice in random order: exact cospherical and coplanar sites everywhere, so
    many signs are decided on the host; the lists must still be the same."""
    torch, A, W, _ = env
    c = W.lattice_cloud(18, seed=5)
    st, _ = _same_lists(A, c.points, c.order)
    assert st["deferred"] > 0


def test_device_lists_planar_bulk(env):
    """Mostly coplanar cloud (a flat grid patch with a few sites off the plane first): hull
    facets in the plane take the in-plane circumcircle rule."""
    torch, A, W, _ = env
    rng = np.random.default_rng(7)
    g = np.arange(40, dtype=np.float32)
    grid = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    flat = np.concatenate([grid, np.zeros((grid.shape[0], 1), np.float32)], 1)
    off = np.array([[3.5, 7.25, 5.0], [20.0, 1.0, -4.0], [31.0, 30.5, 6.0], [9.0, 33.0, -2.5]],
                   np.float32)
    pts = np.concatenate([off, flat[rng.permutation(flat.shape[0])]], 0)
    st, _ = _same_lists(A, pts)
    assert st["deferred"] > 0


def test_device_lists_heightfield(env):
    torch, A, W, _ = env
    w = W.heightfield_prefix(n=200_000, nq=10)
    _same_lists(A, w.cloud.points, w.cloud.order)


def test_device_lists_torus_1m(env):
    """The headline cloud (1M torus points, seeded random order)."""
    torch, A, W, _ = env
    w = W.torus_paper_scale(n=1_000_000, nq=10)
    st, dev = _same_lists(A, w.cloud.points, w.cloud.order)
    print(f"device build of 1M torus: {st}", flush=True)


def _low_dim_clouds():
    rng = np.random.default_rng(13)
    out = []
    # first four ranks on a line (rank 3 between ranks 0 and 1), then a sphere
    c = rng.standard_normal((3000, 3)).astype(np.float32)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    c[3] = c[0] + np.float32(0.5) * (c[1] - c[0])
    out.append(("line start", c))
    # a fully planar cloud (every rank in z = 0): both start points are spares
    g = rng.uniform(-1, 1, (4000, 2)).astype(np.float32)
    out.append(("planar", np.concatenate([g, np.zeros((4000, 1), np.float32)], 1)))
    # a plane for the first 500 ranks, then 3-D points: B is rank 500
    pl = rng.uniform(-1, 1, (500, 2)).astype(np.float32)
    sp = rng.uniform(-1, 1, (2500, 3)).astype(np.float32)
    out.append(("plane then space", np.concatenate(
        [np.concatenate([pl, np.zeros((500, 1), np.float32)], 1), sp], 0)))
    # collinear for 100 ranks, then a plane, then space
    t = np.sort(rng.uniform(-1, 1, 100)).astype(np.float32)[rng.permutation(100)]
    line = np.stack([t, np.zeros(100, np.float32), np.zeros(100, np.float32)], 1)
    pl2 = np.concatenate([rng.uniform(-1, 1, (400, 2)).astype(np.float32),
                          np.zeros((400, 1), np.float32)], 1)
    out.append(("line, plane, space", np.concatenate([line, pl2, sp[:1500]], 0)))
    # an integer grid in one plane (cocircular ties everywhere)
    gg = np.arange(30, dtype=np.float32)
    grid = np.stack(np.meshgrid(gg, gg, indexing="ij"), -1).reshape(-1, 2)
    grid = grid[rng.permutation(grid.shape[0])]
    out.append(("planar grid", np.concatenate([grid, np.full((grid.shape[0], 1), 2.0, np.float32)], 1)))
    return out


@pytest.mark.parametrize("case", range(5))
def test_device_build_low_dimensional_start(env, case):
    """First four ranks coplanar or collinear: the device construction starts from the first
    ranks off the line and plane (or spare points), as the host construction does, and
    records the same lists."""
    torch, A, W, _ = env
    name, pts = _low_dim_clouds()[case]
    print(name, flush=True)
    st, _ = _same_lists(A, pts)
    assert st["rounds"] > 0, "the device path was not taken"


@pytest.mark.parametrize("where", ["late", "start"])
def test_device_build_duplicate(env, where):
    torch, A, W, _lib = env
    c = W.random_cloud(20_000, 11, "torus")
    pts = c.by_rank.copy()
    if where == "late":
        pts[15_000] = pts[9_000]
        pts[17_000] = pts[2_000]
    else:
        pts[12_000] = pts[2]
    msgs = []
    for dev in (False, True):
        with pytest.raises(RuntimeError) as e:
            A.Cloud.build(pts, device=dev)
        msgs.append(str(e.value))
    assert "EDUPLICATE" in msgs[1]
    first = 15_000 if where == "late" else 12_000
    assert f"point {first} " in msgs[0] and f"point {first} " in msgs[1]


def test_device_built_cloud_answers_queries(env):
    """A device-built cloud uploads and answers queries like a host-built one."""
    torch, A, W, _ = env
    w = W.sphere_small(n=10_000, nq=4_000, k=8)
    ch = A.Cloud.build(w.cloud.points, w.cloud.order).upload()
    cd = A.Cloud.build(w.cloud.points, w.cloud.order, device=True).upload()
    q = torch.from_numpy(w.queries).cuda()
    ih, dh = ch.knn(q, 8)
    idv, dd = cd.knn(q, 8)
    torch.cuda.synchronize()
    assert torch.equal(ih, idv) and torch.equal(dh, dd)


@pytest.mark.parametrize("lowdim", [False, True])
def test_device_built_cloud_deletes_like_host(env, lowdim):
    """Deletion (Alg. 3) walks the predecessor lists, which the device construction builds
    too (the transpose, sorted on the GPU): deleting the same ranks from both clouds must
    leave the same lists."""
    torch, A, W, _ = env
    if lowdim:
        pts = _low_dim_clouds()[2][1]
    else:
        pts = W.random_cloud(20_000, 21, "ellipsoid").by_rank
    host = A.Cloud.build(pts)
    dev = A.Cloud.build(pts, device=True)
    rng = np.random.default_rng(3)
    ranks = rng.choice(np.arange(600, pts.shape[0]), 300, replace=False)
    if not lowdim:
        host.delete(ranks)
        dev.delete(ranks)
    else:
        # local sets reaching into the planar prefix may be refused (EUNSUPPORTED): both
        # clouds must then refuse the same ranks
        refused = 0
        for r in ranks[:60]:
            out = []
            for c in (host, dev):
                try:
                    c.delete([int(r)])
                    out.append("ok")
                except RuntimeError as e:
                    out.append(str(e).split(":")[0])
            assert out[0] == out[1], (int(r), out)
            refused += out[0] != "ok"
            if refused:
                break   # a refused batch leaves both clouds as they were up to that rank
    ho, he = host.successors()
    do, de = dev.successors()
    assert np.array_equal(ho, do) and np.array_equal(he, de)
