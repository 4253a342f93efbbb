"""Insertion on the host: appending sites as the newest ranks must leave the lists the
construction of Sec. 3 gives for the live sites plus the new ones, inserted in rank order
(the new ones last).  Combined with deletions (Alg. 3), the reference is the oracle's lists
of the surviving sites and the appended ones, kept in rank order."""
import numpy as np
import pytest

from oracle import successors as S
from oracle import dpknn


@pytest.fixture(scope="module")
def api():
    import os
    from paper_2605_02224_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmknn.so not built")
    from paper_2605_02224_amd import api as A
    return A


def _expected_lists(P, keep):
    """Oracle lists of P[keep] (kept in rank order), mapped back to the ranks of P."""
    Lk = S.successor_lists(P[keep])
    out = [[] for _ in range(P.shape[0])]
    for a, lst in enumerate(Lk):
        out[keep[a]] = [int(keep[b]) for b in lst]
    return out


@pytest.mark.parametrize("seed,shape", [(0, "sphere"), (1, "torus"), (2, "ellipsoid")])
def test_insert_equals_oracle_of_extended_set(api, seed, shape):
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(32, seed=seed, shape=shape, noise=2e-2).by_rank
    cl = api.Cloud.build(P[:20])
    for lo, hi in ((20, 21), (21, 26), (26, 32)):
        got = cl.insert(P[lo:hi])
        assert list(got) == list(range(lo, hi))
        assert cl.n == hi and cl.live_count == hi
        assert cl.lists() == _expected_lists(P[:hi], np.arange(hi)), (lo, hi)


@pytest.mark.parametrize("seed", [3, 4])
def test_delete_then_insert_equals_oracle(api, seed):
    """Deletions drop the kept triangulation; the next insertion must rebuild it from the
    live sites only, so a new site is linked to no deleted one."""
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(36, seed=seed, shape="torus", noise=2e-2).by_rank
    cl = api.Cloud.build(P[:24])
    alive = np.zeros(36, bool)
    alive[:24] = True
    rng = np.random.default_rng(seed)
    cl.insert(P[24:28])          # the triangulation is kept from here on
    alive[24:28] = True
    for step, batch in enumerate(([0, 3], list(rng.choice(np.arange(4, 28), 5, replace=False)))):
        cl.delete(batch)
        alive[batch] = False
        lo, hi = 28 + 4 * step, 32 + 4 * step
        cl.insert(P[lo:hi])
        alive[lo:hi] = True
        keep = np.flatnonzero(alive)
        assert cl.lists()[:hi] == _expected_lists(P[:hi], keep), step
        assert cl.head == int(keep[0]) and cl.live_count == keep.size


def test_insert_reuses_deleted_coordinates(api):
    """A deleted site's position is free: a new site may take it (a new rank)."""
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(24, seed=5, shape="sphere", noise=2e-2).by_rank
    cl = api.Cloud.build(P)
    cl.delete([7])
    cl.insert(P[7:8])
    Q = np.concatenate([P, P[7:8]])
    keep = np.array([r for r in range(25) if r != 7])
    assert cl.lists() == _expected_lists(Q, keep)


def test_insert_errors_leave_cloud_unchanged(api):
    from paper_2605_02224_amd import _lib
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(24, seed=6, shape="torus", noise=2e-2).by_rank
    cl = api.Cloud.build(P[:20])
    before = cl.lists()
    new = P[20:24].copy()
    for bad, status in ((np.concatenate([new, P[5:6]]), _lib.EDUPLICATE),       # a live site
                        (np.concatenate([new, new[1:2]]), _lib.EDUPLICATE),     # within the batch
                        (np.where(np.arange(12).reshape(4, 3) == 7, np.nan, new), _lib.ENONFINITE)):
        with pytest.raises(_lib.MknnError) as e:
            cl.insert(bad)
        assert e.value.status == status
        assert cl.n == 20 and cl.lists() == before
    cl.insert(new)
    assert cl.lists() == _expected_lists(P, np.arange(24))


def test_insert_needs_four_live_sites(api):
    from paper_2605_02224_amd import _lib
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(12, seed=7, shape="sphere", noise=2e-2).by_rank
    cl = api.Cloud.build(P[:6])
    cl.delete([0, 1, 2])
    with pytest.raises(_lib.MknnError) as e:
        cl.insert(P[6:8])
    assert e.value.status == _lib.EUNSUPPORTED
    assert cl.n == 6


def test_insert_3000_equals_build_and_brute_force(api):
    """Growing 2400 points to 3000 in batches equals building the 3000 points, and the
    prefix k-NN over the grown lists equals brute force."""
    import oracle
    oracle.build(force=False)
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(3000, seed=8, shape="torus").by_rank
    cl = api.Cloud.build(P[:2400])
    for b in range(2400, 3000, 150):
        cl.insert(P[b:b + 150])
    ref = api.Cloud.build(P).lists()
    got = cl.lists()
    assert got == ref
    lo, hi = W.bbox_expanded(P, 1.1)
    Q = W.uniform_in_box(np.random.default_rng(2), 200, lo, hi)
    for k, m in ((10, 3000), (5, 2600)):
        ri, _, _ = oracle.knn_bruteforce(P, Q, k, m)
        idx, _, _, _ = dpknn.dp_knn_batch(P, got, Q, k, m, head=cl.head)
        assert (idx == ri).all()
