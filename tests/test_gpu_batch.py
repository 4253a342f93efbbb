"""GPU parity of the batched form: many clouds in one launch per class, against
the oracle and bit-for-bit against the plain per-cloud launch."""
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
    rng = np.random.default_rng(42)
    clouds = []
    for i in range(18):
        n = int(np.exp(rng.uniform(np.log(300), np.log(40000))))
        c = W.random_cloud(n, seed=100 + i, shape=W.SHAPES[i % 3])
        P = c.by_rank
        clouds.append((P, A.Cloud.build(P).upload()))
    return torch, oracle, A, W, clouds


def _make_batch(env, seed, k_choices=(1, 4, 10, 16, 17, 33, 64)):
    torch, oracle, A, W, clouds = env
    rng = np.random.default_rng(seed)
    items, host = [], []
    for i, (P, cl) in enumerate(clouds):
        if rng.uniform() < 0.15:
            continue
        nq = int(rng.choice([0, 1, 37, 500, 3000, 9000]))
        k = int(rng.choice(k_choices))
        m = 0 if rng.uniform() < 0.5 else int(rng.integers(1, P.shape[0] + 1))
        lo, hi = W.bbox_expanded(P, 1.05)
        Q = W.uniform_in_box(rng, nq, lo, hi)
        items.append((cl, torch.from_numpy(Q).cuda(), k, m))
        host.append((P, Q, k, m))
    return A.alloc_outputs(items), host


def _check(env, items, host, sample=400):
    torch, oracle, A, W, clouds = env
    rng = np.random.default_rng(0)
    ex = 0
    for (cl, q, k, m, idx, dist), (P, Q, _, _) in zip(items, host):
        if Q.shape[0] == 0:
            continue
        mm = P.shape[0] if m == 0 else m
        sel = rng.choice(Q.shape[0], min(sample, Q.shape[0]), replace=False)
        ri, _, rD = oracle.knn_bruteforce(P, Q[sel], k + 1, mm)
        ex += compare_rows(idx.cpu().numpy()[sel], dist.cpu().numpy()[sel], ri[:, :k],
                           rD[:, :k], rD[:, k], P=P, Q=Q[sel], m=mm)
    return ex


@pytest.mark.parametrize("sort,graph", [(True, True), (False, True), (True, False)])
def test_batch_matches_oracle_and_plain(env, sort, graph):
    torch, oracle, A, W, clouds = env
    items, host = _make_batch(env, seed=1)
    plan = A.BatchPlan(64, 200000, tile_queries=256, sort=sort, graph=graph)
    plan.run(items)
    torch.cuda.synchronize()
    assert _check(env, items, host) <= 3
    # the plain launch runs the same per-query walk: identical bits
    for cl, q, k, m, idx, dist in items:
        if q.shape[0] == 0:
            continue
        pi, pd = cl.knn(q, k, None if m == 0 else m)
        assert torch.equal(pi, idx) and torch.equal(pd, dist)


@pytest.mark.parametrize("graph", [True, False])
def test_persistent_launch_matches_plain(env, graph):
    """The persistent tile-claiming launch (chosen at plan creation by MKNN_BATCH_PERSISTENT)
    gives the plain launch's bits, like the default flat launch."""
    import os
    torch, oracle, A, W, clouds = env
    items, host = _make_batch(env, seed=3)
    os.environ["MKNN_BATCH_PERSISTENT"] = "1"
    try:
        plan = A.BatchPlan(64, 200000, tile_queries=16, sort=True, graph=graph)
    finally:
        del os.environ["MKNN_BATCH_PERSISTENT"]
    for rep in range(2):
        plan.run(items)
        torch.cuda.synchronize()
        for cl, q, k, m, idx, dist in items:
            if q.shape[0] == 0:
                continue
            pi, pd = cl.knn(q, k, None if m == 0 else m)
            assert torch.equal(pi, idx) and torch.equal(pd, dist)
    assert _check(env, items, host, sample=200) <= 3


def test_graph_replays_with_changing_batches(env):
    """One captured graph replays different batches; between replays the program does its
    own eager work and synchronises; every replay equals the eager result."""
    torch, oracle, A, W, clouds = env
    plan = A.BatchPlan(64, 200000, tile_queries=512, sort=True, graph=True)
    eager = A.BatchPlan(64, 200000, tile_queries=512, sort=True, graph=False)
    for rep in range(4):
        items, host = _make_batch(env, seed=10 + rep)
        plan.run(items)
        torch.cuda.synchronize()
        got = [(i.clone(), d.clone()) for (_, _, _, _, i, d) in items]
        _ = torch.randn(1000, device="cuda").sum().item()      # unrelated eager work
        eager.run(items)
        torch.cuda.synchronize()
        for (gi, gd), (_, _, _, _, i, d) in zip(got, items):
            assert torch.equal(gi, i) and torch.equal(gd, d)
        if rep == 0:
            assert _check(env, items, host, sample=200) <= 3


def test_convenience_entry_and_empty(env):
    torch, oracle, A, W, clouds = env
    A.batch_knn([])
    items, host = _make_batch(env, seed=5, k_choices=(10,))
    A.batch_knn(items)
    torch.cuda.synchronize()
    assert _check(env, items, host, sample=200) <= 3


def test_batch_errors(env):
    torch, oracle, A, W, clouds = env
    from paper_2605_02224_amd._lib import MknnError
    P, cl = clouds[0]
    q = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    plan = A.BatchPlan(2, 100, tile_queries=16)
    with pytest.raises(MknnError):
        plan.run(A.alloc_outputs([(cl, q, 65, 0)]))
    with pytest.raises(MknnError):
        plan.run(A.alloc_outputs([(cl, q, 4, P.shape[0] + 1)]))
    with pytest.raises(MknnError):
        plan.run(A.alloc_outputs([(cl, q, 4, 0)] * 3))          # over request capacity
    big = torch.zeros((101, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(MknnError):
        plan.run(A.alloc_outputs([(cl, big, 4, 0)]))            # over query capacity


def test_256_clouds_paper_scale_sampled(env):
    """Batched form at full size: 256 clouds, sizes log-uniform in [1e3, 2e5] (about 10M
    points), 4 n_c queries each, k=10, one batch in the launch configuration the benchmark
    times (default 16-query tiles, sorted, graph), checked on a sample of every cloud's rows."""
    torch, oracle, A, W, _ = env
    import concurrent.futures as cf
    w = W.many_clouds()
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        built = list(ex.map(lambda c: A.Cloud.build(c.by_rank), w.clouds))
    for cl in built:
        cl.upload()
    items = A.alloc_outputs([(cl, torch.from_numpy(q).cuda(), w.k, None)
                             for cl, q in zip(built, w.queries)])
    plan = A.BatchPlan(len(items), sum(it[1].shape[0] for it in items))
    plan.run(items)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    exc = rows = 0
    # 16 clouds in full, 2,000 sampled rows of every other cloud
    whole = set(rng.choice(len(items), 16, replace=False).tolist())
    for i, (c, (cl, q, k, m, idx, dist)) in enumerate(zip(w.clouds, items)):
        Qa = q.cpu().numpy()
        sel = (np.arange(Qa.shape[0]) if i in whole else
               rng.choice(Qa.shape[0], min(2000, Qa.shape[0]), replace=False))
        ri, _, rD = oracle.knn_bruteforce(c.by_rank, Qa[sel], k + 1)
        exc += compare_rows(idx.cpu().numpy()[sel], dist.cpu().numpy()[sel], ri[:, :k], rD[:, :k],
                            rD[:, k], P=c.by_rank, Q=Qa[sel])
        rows += sel.size
    print(f"256 clouds: {rows} rows checked, near-ties excused {exc}")
    assert exc <= 6
    plan.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_waves_moving_between_clouds_of_very_different_size(env, persistent):
    """Wavefronts take tiles of one request after another; rows idle at a switch still hold
    the descriptor of the previous request's cloud, which must never be used to address the
    next cloud's (much smaller) arena.  Tiny clouds interleaved with a large one, small
    tiles, and every result checked against the oracle -- in the default flat launch and in
    the persistent tile-claiming launch, where a wavefront does change request."""
    import os
    torch, oracle, A, W, clouds = env
    rng = np.random.default_rng(41)
    big = W.random_cloud(120000, seed=42, shape="torus").by_rank
    parts = [(big, A.Cloud.build(big).upload())]
    for i in range(12):
        P = W.random_cloud(int(rng.integers(8, 40)), seed=60 + i, shape=W.SHAPES[i % 3]).by_rank
        parts.append((P, A.Cloud.build(P).upload()))
    items, host = [], []
    for rep in range(3):
        for P, cl in parts:
            nq = 3000 if P.shape[0] > 1000 else 64
            k = int(rng.choice([4, 16, 24]))
            Q = W.uniform_in_box(rng, nq, *W.bbox_expanded(P, 1.1))
            items.append((cl, torch.from_numpy(Q).cuda(), k, 0))
            host.append((P, Q, k, 0))
    items = A.alloc_outputs(items)
    if persistent:
        os.environ["MKNN_BATCH_PERSISTENT"] = "1"
    try:
        plan = A.BatchPlan(len(items), 20000, tile_queries=4, sort=True, graph=False)
    finally:
        os.environ.pop("MKNN_BATCH_PERSISTENT", None)
    plan.run(items)
    torch.cuda.synchronize()
    assert _check(env, items, host) <= 3
