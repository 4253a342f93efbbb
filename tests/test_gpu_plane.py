"""GPU k-NN with a local plane fit per row (the scan convergence statistic, Sec. 5.3.1)
against the oracle: brute-force rows, then the reference PCA fit (oracle/planefit.py) on the
oracle's neighbours."""
import numpy as np
import pytest

from tests._compare import compare_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    oracle.build(force=False)
    from oracle import planefit
    from paper_2605_02224_amd import api as A
    from paper_2605_02224_amd import workloads as W
    return torch, oracle, planefit, A, W


def _check_planes(P, gi, ri, got, ref):
    """Compare planes on rows whose neighbour sets agree with the oracle's."""
    same = np.array([set(a[a >= 0]) == set(b[b >= 0]) for a, b in zip(gi, ri)])
    assert same.mean() > 0.99
    got, ref = got[same].astype(np.float64), ref[same]
    scale = np.abs(P).max()
    defined = ~np.isnan(ref[:, 3])
    assert (np.isnan(got[:, 3:]) == np.isnan(ref[:, 3:])).all()
    cdef = ~np.isnan(ref[:, 0])
    assert (np.isnan(got[:, 0]) == ~cdef).all()
    assert np.allclose(got[cdef, :3], ref[cdef, :3], rtol=0, atol=2e-6 * scale)
    if not defined.any():
        return 0
    g, r = got[defined], ref[defined]
    # the normal is well defined where the two smallest eigenvalues are apart; the sign rule
    # is stable where the largest component leads the others clearly
    dot = np.abs((g[:, 3:6] * r[:, 3:6]).sum(axis=1))
    lam0 = r[:, 6] ** 2
    spread = np.array([np.linalg.eigvalsh(np.cov(P[i[i >= 0]].T.astype(np.float64), bias=True))
                       for i in ri[same][defined]])
    gap = (spread[:, 1] - spread[:, 0]) / np.maximum(spread[:, 2], 1e-300)
    ok = gap > 1e-3
    assert (dot[ok] > 1 - 1e-5).all(), dot[ok].min()
    comp = np.sort(np.abs(r[:, 3:6]), axis=1)
    clear = ok & (comp[:, 2] - comp[:, 1] > 1e-4)
    assert np.allclose(g[clear, 3:6], r[clear, 3:6], atol=1e-4)
    # residual: absolute error of lambda_0 ~ 1e-15 lambda_2 in float64, then float32 output
    tol = 2e-7 * np.sqrt(spread[:, 2]) + 2e-6 * r[:, 6]
    assert (np.abs(g[:, 6] - r[:, 6]) <= tol).all()
    assert np.allclose(g[:, 7], r[:, 7], rtol=1e-4, atol=1e-6)
    return int(defined.sum())


@pytest.mark.parametrize("shape,k,m", [("torus", 20, None), ("sphere", 16, None),
                                       ("ellipsoid", 40, 9000), ("torus", 20, 2)])
def test_plane_fit_rows(env, shape, k, m):
    torch, oracle, planefit, A, W = env
    c = W.random_cloud(20000, seed=31, shape=shape)
    P = c.by_rank
    cl = A.Cloud.build(P).upload()
    rng = np.random.default_rng(5)
    # probes near the surface (the scan convergence setting) and volume queries
    near = P[rng.choice(P.shape[0], 3000)] + rng.normal(0, 1e-3, (3000, 3)).astype(np.float32)
    Q = np.concatenate([near, W.uniform_in_box(rng, 2000, *W.bbox_expanded(P, 1.1))])
    idx, dist, plane = cl.knn_plane(torch.from_numpy(Q).cuda(), k, m)
    torch.cuda.synchronize()
    gi, gd, gp = idx.cpu().numpy(), dist.cpu().numpy(), plane.cpu().numpy()
    ri, _, rD = oracle.knn_bruteforce(P, Q, k + 1, m)
    ex = compare_rows(gi, gd, ri[:, :k], rD[:, :k], rD[:, k], P=P, Q=Q, m=m)
    assert ex <= 2
    # the same rows as the plain query
    i2, d2 = cl.knn(torch.from_numpy(Q).cuda(), k, m)
    assert (i2.cpu().numpy() == gi).all() and (d2.cpu().numpy() == gd).all()
    ref = planefit.plane_fit_rows(P, ri[:, :k])
    fitted = _check_planes(P, gi, ri[:, :k], gp, ref)
    if m == 2:
        assert fitted == 0 and np.isnan(gp[:, 3:]).all()
    else:
        assert fitted == Q.shape[0]


def test_plane_fit_after_insertion(env):
    """Appended points reach the per-rank point array the fit reads."""
    torch, oracle, planefit, A, W = env
    P = W.random_cloud(12000, seed=32, shape="sphere").by_rank
    cl = A.Cloud.build(P[:10000]).upload()
    cl.insert(P[10000:])
    rng = np.random.default_rng(6)
    Q = P[10000 + rng.choice(2000, 1000)] + rng.normal(0, 1e-3, (1000, 3)).astype(np.float32)
    idx, dist, plane = cl.knn_plane(torch.from_numpy(Q).cuda(), 20)
    torch.cuda.synchronize()
    ri, _, rD = oracle.knn_bruteforce(P, Q, 21)
    gi = idx.cpu().numpy()
    ex = compare_rows(gi, dist.cpu().numpy(), ri[:, :20], rD[:, :20], rD[:, 20], P=P, Q=Q)
    assert ex <= 2
    _check_planes(P, gi, ri[:, :20], plane.cpu().numpy(), planefit.plane_fit_rows(P, ri[:, :20]))
