"""GPU queries after deletions: device lists updated by copy-on-write deltas answer k-NN
over the surviving prefix exactly (Sec. 4.3)."""
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
    from paper_2605_02224_amd import api as A
    from paper_2605_02224_amd import workloads as W
    return torch, oracle, A, W


def _check(env, cl, P, live, Q, k, m=None):
    torch, oracle, A, W = env
    idx, dist = cl.knn(torch.from_numpy(Q).cuda(), k, m)
    torch.cuda.synchronize()
    ri, _, rD = oracle.knn_bruteforce(P, Q, k + 1, m, live=live)
    return compare_rows(idx.cpu().numpy(), dist.cpu().numpy(), ri[:, :k], rD[:, :k], rD[:, k],
                        P=P, Q=Q, m=m, live=live)


def test_queries_after_deletion_batches(env):
    torch, oracle, A, W = env
    c = W.random_cloud(40000, seed=21, shape="ellipsoid")
    P = c.by_rank
    cl = A.Cloud.build(P).upload()
    live = np.ones(40000, np.uint8)
    rng = np.random.default_rng(3)
    lo, hi = W.bbox_expanded(P, 1.1)
    Q = W.uniform_in_box(rng, 12000, lo, hi)
    order = rng.permutation(40000)
    dead = np.concatenate([[0, 1, 2], order[:2000]])
    dead = dead[np.sort(np.unique(dead, return_index=True)[1])]
    for b in range(0, dead.size, 500):
        cl.delete(dead[b:b + 500])
        live[dead[b:b + 500]] = 0
        for k, m in ((16, None), (8, 25000), (33, None)):
            assert _check(env, cl, P, live, Q, k, m) <= 2
    assert cl.head == int(np.flatnonzero(live)[0])


def test_copy_on_write_keeps_earlier_work_on_the_old_lists(env):
    """A query batch enqueued before a deletion on the same stream answers on the old
    lists; one enqueued after answers on the new lists."""
    torch, oracle, A, W = env
    c = W.random_cloud(20000, seed=22, shape="torus")
    P = c.by_rank
    cl = A.Cloud.build(P).upload()
    lo, hi = W.bbox_expanded(P, 1.1)
    Q = W.uniform_in_box(np.random.default_rng(4), 50000, lo, hi)
    qd = torch.from_numpy(Q).cuda()
    before = cl.knn(qd, 10)                       # enqueued, not yet synchronised
    dead = np.random.default_rng(5).choice(20000, 1000, replace=False)
    cl.delete(dead)                               # same (current) stream
    after = cl.knn(qd, 10)
    torch.cuda.synchronize()
    live = np.ones(20000, np.uint8)
    ri, _, rD = oracle.knn_bruteforce(P, Q[:2000], 10)
    ex = compare_rows(before[0].cpu().numpy()[:2000], before[1].cpu().numpy()[:2000], ri, rD,
                      P=P, Q=Q[:2000])
    live[dead] = 0
    ri, _, rD = oracle.knn_bruteforce(P, Q[:2000], 10, live=live)
    ex += compare_rows(after[0].cpu().numpy()[:2000], after[1].cpu().numpy()[:2000], ri, rD,
                       P=P, Q=Q[:2000], live=live)
    assert ex <= 2


def test_repack_when_slack_runs_out(env):
    """Deleting most of a small cloud exhausts the arena slack and triggers a full re-pack."""
    torch, oracle, A, W = env
    c = W.random_cloud(3000, seed=23, shape="sphere")
    P = c.by_rank
    cl = A.Cloud.build(P).upload()
    live = np.ones(3000, np.uint8)
    rng = np.random.default_rng(6)
    Q = W.uniform_in_box(rng, 3000, *W.bbox_expanded(P, 1.2))
    dead = rng.permutation(3000)[:2500]
    for b in range(0, 2500, 250):
        cl.delete(dead[b:b + 250])
        live[dead[b:b + 250]] = 0
        assert _check(env, cl, P, live, Q, 12) <= 2


def test_compact_after_deletions_keeps_results(env):
    """Re-packing the device lists after deletions gives back the slack and changes no
    result bit."""
    torch, oracle, A, W = env
    c = W.random_cloud(20000, seed=24, shape="ellipsoid")
    P = c.by_rank
    cl = A.Cloud.build(P).upload()
    rng = np.random.default_rng(8)
    dead = rng.choice(20000, 600, replace=False)
    for b in range(0, 600, 200):
        cl.delete(dead[b:b + 200])
    Q = W.uniform_in_box(rng, 20000, *W.bbox_expanded(P, 1.1))
    qd = torch.from_numpy(Q).cuda()
    before = cl.knn(qd, 20)
    torch.cuda.synchronize()
    cl.compact()
    after = cl.knn(qd, 20)
    torch.cuda.synchronize()
    assert torch.equal(before[0], after[0]) and torch.equal(before[1], after[1])
    live = np.ones(20000, np.uint8)
    live[dead] = 0
    ri, _, rD = oracle.knn_bruteforce(P, Q[:1500], 21, live=live)
    ex = compare_rows(after[0].cpu().numpy()[:1500], after[1].cpu().numpy()[:1500], ri[:, :20],
                      rD[:, :20], rD[:, 20], P=P, Q=Q[:1500], live=live)
    assert ex <= 2


def test_queries_after_insertions_and_deletions(env):
    """Points appended on the device (copy-on-write list segments and new descriptors, then
    a re-pack once the descriptor slack runs out) answer k-NN over the grown cloud and over
    prefixes that end before, at and after the appended ranks."""
    torch, oracle, A, W = env
    c = W.random_cloud(26000, seed=23, shape="torus")
    P = c.by_rank
    n0 = 20000
    cl = A.Cloud.build(P[:n0]).upload()
    live = np.ones(26000, np.uint8)
    rng = np.random.default_rng(5)
    lo, hi = W.bbox_expanded(P, 1.1)
    Q = W.uniform_in_box(rng, 10000, lo, hi)
    n = n0
    for step, cnt in enumerate((1000, 1500, 1500, 2000)):   # the third batch outgrows the slack
        if step == 2:
            dead = rng.choice(n, 300, replace=False)
            cl.delete(dead)
            live[dead] = 0
        assert list(cl.insert(P[n:n + cnt])) == list(range(n, n + cnt))
        n += cnt
        assert cl.n == n
        for k, m in ((16, None), (8, n - cnt // 2), (33, n0 - 10)):
            assert _check(env, cl, P[:n], live[:n], Q, k, m) <= 2, (step, k, m)
