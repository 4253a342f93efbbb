"""Deletion (Alg. 3) on the host: the lists after deleting a set D must equal the lists of
P \\ D inserted in the original relative order (Sec. 4.3)."""
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
    """Oracle lists of P[keep] (kept in rank order), mapped back to original ranks."""
    Lk = S.successor_lists(P[keep])
    out = [[] for _ in range(P.shape[0])]
    for a, lst in enumerate(Lk):
        out[keep[a]] = [int(keep[b]) for b in lst]
    return out


@pytest.mark.parametrize("seed,shape", [(0, "sphere"), (1, "torus"), (2, "ellipsoid"),
                                        (3, "torus")])
def test_delete_equals_oracle_rebuild(api, seed, shape):
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(30, seed=seed, shape=shape, noise=2e-2).by_rank
    cl = api.Cloud.build(P)
    rng = np.random.default_rng(seed)
    alive = np.ones(30, bool)
    # head first, then the next oldest ranks (the low-dimensional start), then random ones
    plan = [[0], [1], [2, 5], list(rng.choice(np.arange(6, 30), 6, replace=False))]
    for batch in plan:
        before = cl.lists()
        cl.delete(batch)
        alive[batch] = False
        keep = np.flatnonzero(alive)
        after = cl.lists()
        assert after == _expected_lists(P, keep), batch
        # Lemma 1: no entry between surviving sites disappears
        for i in keep:
            assert set(j for j in before[i] if alive[j]) <= set(after[i])
        assert cl.head == int(keep[0]) and cl.live_count == keep.size


def test_delete_equals_build_of_remaining_3000(api):
    """Deleting 10% of 3000 points in batches equals building the remaining points."""
    import oracle
    oracle.build(force=False)
    from paper_2605_02224_amd import workloads as W
    c = W.random_cloud(3000, seed=4, shape="torus")
    P = c.by_rank
    cl = api.Cloud.build(P)
    rng = np.random.default_rng(1)
    dead = rng.choice(3000, 300, replace=False)
    for b in range(0, 300, 100):
        cl.delete(dead[b:b + 100])
    keep = np.setdiff1d(np.arange(3000), dead)
    ref = api.Cloud.build(P[keep]).lists()
    got = cl.lists()
    mapped = [[] for _ in range(3000)]
    for a, lst in enumerate(ref):
        mapped[keep[a]] = [int(keep[x]) for x in lst]
    assert got == mapped
    # k-NN over the surviving prefix by walking the edited lists equals brute force
    live = np.zeros(3000, np.uint8)
    live[keep] = 1
    lo, hi = W.bbox_expanded(P, 1.1)
    Q = W.uniform_in_box(np.random.default_rng(2), 200, lo, hi)
    for k, m in ((10, 3000), (4, 1700)):
        ri, _, rD = oracle.knn_bruteforce(P, Q, k, m, live=live)
        idx, D, _, _ = dpknn.dp_knn_batch(P, got, Q, k, m, head=cl.head)
        assert (idx == ri).all()


def test_delete_errors_are_atomic(api):
    from paper_2605_02224_amd._lib import MknnError, ENOTFOUND, EINVAL
    rng = np.random.default_rng(0)
    P = rng.standard_normal((40, 3)).astype(np.float32)
    cl = api.Cloud.build(P)
    cl.delete([5])
    before = cl.lists()
    for bad in ([5], [3, 3], [-1], [40], [7, 5]):
        with pytest.raises(MknnError) as e:
            cl.delete(bad)
        assert e.value.status == ENOTFOUND
        assert cl.lists() == before
    with pytest.raises(MknnError) as e:
        cl.delete([i for i in range(40) if i != 5])
    assert e.value.status == EINVAL


@pytest.mark.parametrize("seed", range(8))
def test_delete_one_at_a_time_random(api, seed):
    """Delete half of a 24-point cloud one rank at a time in random order; after every step
    the lists equal the exact lists of the survivors."""
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(24, seed=50 + seed, shape=W.SHAPES[seed % 3], noise=3e-2).by_rank
    cl = api.Cloud.build(P)
    alive = np.ones(24, bool)
    for r in np.random.default_rng(seed).permutation(24)[:12]:
        cl.delete([int(r)])
        alive[r] = False
        assert cl.lists() == _expected_lists(P, np.flatnonzero(alive)), int(r)


@pytest.mark.parametrize("frac", [0.05, 0.4])
def test_batch_in_rounds_equals_build_of_remaining(api, frac):
    """One large batch is reordered into rounds of independent deletions, each round's
    redistributions on several threads; the lists equal a build of the remaining points
    (Sec. 4.3), also when many deleted ranks are neighbours of each other (40% deleted,
    many rounds) and when the head and the oldest ranks are in the batch."""
    from paper_2605_02224_amd import workloads as W
    n = 6000
    P = W.random_cloud(n, seed=9, shape="sphere").by_rank
    cl = api.Cloud.build(P)
    rng = np.random.default_rng(3)
    dead = rng.choice(n, int(frac * n), replace=False)
    dead = np.unique(np.concatenate([dead, [0, 1, 2, 7]]))
    rng.shuffle(dead)
    cl.delete(dead)
    keep = np.setdiff1d(np.arange(n), dead)
    ref = api.Cloud.build(P[keep]).lists()
    mapped = [[] for _ in range(n)]
    for a, lst in enumerate(ref):
        mapped[keep[a]] = [int(keep[x]) for x in lst]
    assert cl.lists() == mapped
    assert cl.live_count == keep.size and cl.head == int(keep[0])
