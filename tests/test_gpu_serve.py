"""GPU tests of the serving loop: continuous batching over resident clouds with deletions
between batches (Sec. 4.3).  Every request must return, bit for bit, what it returns when
run alone, and requests on either side of a deletion must see the lists before / after it."""
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


def _clouds(env, count, seed, nmax=30000):
    torch, oracle, A, W = env
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(500), np.log(nmax))))
        P = W.random_cloud(n, seed=seed * 100 + i, shape=W.SHAPES[i % 3]).by_rank
        out.append((P, A.Cloud.build(P).upload()))
    torch.cuda.synchronize()
    return out


def _requests(env, clouds, count, seed):
    torch, oracle, A, W = env
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(count):
        c = int(rng.integers(len(clouds)))
        P, cl = clouds[c]
        nq = int(rng.choice([1, 17, 256, 1000, 4000]))
        k = int(rng.choice([1, 8, 16, 24, 64]))
        m = None if rng.uniform() < 0.6 else int(rng.integers(1, P.shape[0] + 1))
        Q = W.uniform_in_box(rng, nq, *W.bbox_expanded(P, 1.1))
        reqs.append((c, Q, torch.from_numpy(Q).cuda(), k, m))
    return reqs


@pytest.mark.parametrize("plain", [False, True])
def test_each_result_same_alone_and_in_the_mix(env, plain):
    torch, oracle, A, W = env
    clouds = _clouds(env, 10, seed=1)
    reqs = _requests(env, clouds, 120, seed=2)
    alone = []
    for c, Q, q, k, m in reqs:
        idx, dist = clouds[c][1].knn(q, k, m)
        alone.append((idx, dist))
    torch.cuda.synchronize()
    srv = A.Server(pool_queries=1 << 15, nstreams=2, max_wave_requests=32, plain=plain)
    tickets = [srv.submit(clouds[c][1], q, k, m) for c, Q, q, k, m in reqs]
    got = [srv.wait(t)[2] for t in tickets]
    waves, wreq = srv.stats()
    srv.close()
    assert wreq == len(reqs)
    if plain:
        assert waves == len(reqs)
    else:
        assert waves < len(reqs)          # requests were batched together
    for (c, Q, q, k, m), (ai, ad), bufs in zip(reqs, alone, got):
        assert torch.equal(ai, bufs[1]) and torch.equal(ad, bufs[2])
    # and the mix agrees with the oracle on a sample of every request
    rng = np.random.default_rng(3)
    ex = 0
    for (c, Q, q, k, m), bufs in zip(reqs[:40], got[:40]):
        P = clouds[c][0]
        sel = rng.choice(Q.shape[0], min(64, Q.shape[0]), replace=False)
        ri, _, rD = oracle.knn_bruteforce(P, Q[sel], k + 1, m)
        ex += compare_rows(bufs[1].cpu().numpy()[sel], bufs[2].cpu().numpy()[sel], ri[:, :k],
                           rD[:, :k], rD[:, k], P=P, Q=Q[sel], m=m)
    assert ex <= 2


def test_host_outputs_match_device_outputs(env):
    torch, oracle, A, W = env
    clouds = _clouds(env, 3, seed=4)
    reqs = _requests(env, clouds, 30, seed=5)
    srv = A.Server(pool_queries=1 << 14, nstreams=2, max_wave_requests=8)
    tickets = []
    for c, Q, q, k, m in reqs:
        hi = torch.empty((Q.shape[0], k), dtype=torch.int32).pin_memory()
        hd = torch.empty((Q.shape[0], k), dtype=torch.float32).pin_memory()
        tickets.append(srv.submit(clouds[c][1], q, k, m, h_idx=hi, h_dist=hd))
    for t in tickets:
        _, _, (q, idx, dist, hi, hd) = srv.wait(t)
        assert torch.equal(idx.cpu(), hi) and torch.equal(dist.cpu(), hd)
    srv.close()


@pytest.mark.parametrize("order", ["strict", "bind_at_admission", "lazy_delete"])
def test_deletions_between_batches(env, order):
    """Requests and deletion batches interleaved on several clouds.  Each request reports how
    many deletion batches of its cloud it saw and must equal the oracle on the live set after
    exactly those.  In the strict orders (the default, and its form that filters marked
    deletions instead of waiting for them) that number is the count of deletions submitted
    before the request.  Enough deletions are made on the small cloud to run out of arena
    slack, which forces a full re-pack while other waves are in flight."""
    bind_at_admission = order == "bind_at_admission"
    torch, oracle, A, W = env
    clouds = _clouds(env, 4, seed=6, nmax=20000)
    P0 = W.random_cloud(3000, seed=77, shape="sphere").by_rank
    clouds.append((P0, A.Cloud.build(P0).upload()))
    torch.cuda.synchronize()
    masks = [[np.ones(P.shape[0], np.uint8)] for P, _ in clouds]   # live set after v deletions
    rng = np.random.default_rng(7)
    srv = A.Server(pool_queries=1 << 15, nstreams=2, max_wave_requests=16,
                   bind_at_admission=bind_at_admission, lazy_delete=order == "lazy_delete")
    log = []
    for step in range(70):
        c = int(rng.integers(len(clouds)))
        P, cl = clouds[c]
        live = masks[c][-1]
        if rng.uniform() < 0.3 and live.sum() > 600:
            alive = np.flatnonzero(live)
            cnt = 250 if c == len(clouds) - 1 else int(rng.integers(1, 200))
            dead = rng.choice(alive, min(cnt, alive.size - 500), replace=False)
            if rng.uniform() < 0.3:
                dead = np.unique(np.concatenate([[alive[0]], dead]))   # the head too
            nxt = live.copy()
            nxt[dead] = 0
            masks[c].append(nxt)
            log.append(("del", srv.delete(cl, dead), c, None, None, None))
        else:
            nq = int(rng.choice([50, 500, 2000]))
            k = int(rng.choice([4, 16, 40]))
            Q = W.uniform_in_box(rng, nq, *W.bbox_expanded(P, 1.1))
            t = srv.submit(cl, torch.from_numpy(Q).cuda(), k)
            log.append(("knn", t, c, Q, k, len(masks[c]) - 1))
    res = {t: srv.wait(t, with_seen=True) for _, t, *_ in log}
    srv.close()
    ex = 0
    for kind, t, c, Q, k, before in log:
        if kind != "knn":
            continue
        _, _, (_, idx, dist, *_), seen = res[t]
        if not bind_at_admission:
            assert seen == before
        assert 0 <= seen < len(masks[c])
        P = clouds[c][0]
        sel = np.arange(min(100, Q.shape[0]))
        ri, _, rD = oracle.knn_bruteforce(P, Q[sel], k + 1, live=masks[c][seen])
        ex += compare_rows(idx.cpu().numpy()[sel], dist.cpu().numpy()[sel], ri[:, :k],
                           rD[:, :k], rD[:, k], P=P, Q=Q[sel], live=masks[c][seen])
    assert ex <= 2
    for c, (P, cl) in enumerate(clouds):
        assert cl.live_count == int(masks[c][-1].sum())
        assert cl.head == int(np.flatnonzero(masks[c][-1])[0])


def test_errors_and_empty_requests(env):
    torch, oracle, A, W = env
    from paper_2605_02224_amd._lib import MknnError, EBUSY, EUNSUPPORTED, ENOTFOUND, EINVAL
    (P, cl), = _clouds(env, 1, seed=8, nmax=2000)
    srv = A.Server(pool_queries=1000, nstreams=2, max_wave_requests=4)
    q = torch.zeros((501, 3), device="cuda")
    with pytest.raises(MknnError) as e:
        srv.submit(cl, q, 4)                      # larger than a slot (500 queries)
    assert e.value.status == EBUSY
    with pytest.raises(MknnError) as e:
        srv.submit(cl, q[:10], 65)
    assert e.value.status == EUNSUPPORTED
    with pytest.raises(MknnError) as e:
        srv.submit(cl, q[:10], 4, m=P.shape[0] + 1)
    assert e.value.status == EINVAL
    t = srv.submit(cl, q[:0], 4)
    assert srv.done(t)
    srv.wait(t)
    with pytest.raises(MknnError) as e:
        srv.done(t)
    assert e.value.status == ENOTFOUND
    # a failing deletion reports its error and leaves the cloud as it was
    t = srv.delete(cl, [P.shape[0]])
    with pytest.raises(MknnError) as e:
        srv.wait(t)
    assert e.value.status == ENOTFOUND
    t = srv.submit(cl, torch.from_numpy(P[:5]).cuda(), 1)
    _, _, (_, idx, dist, *_) = srv.wait(t)
    assert idx.cpu().numpy()[:, 0].tolist() == list(range(5))
    assert (dist.cpu().numpy() == 0).all()
    srv.close()


@pytest.mark.parametrize("mode", ["batched", "plain", "lazy_delete"])
def test_insertions_and_deletions_between_batches(env, mode):
    """Insertion batches go through the same ordered update path as deletions: every
    request sees exactly the update batches submitted before it on its cloud, and equals
    the oracle on the points present after those (new points take the next ranks)."""
    torch, oracle, A, W = env
    Pfull = [W.random_cloud(n, seed=90 + i, shape=W.SHAPES[i % 3]).by_rank
             for i, n in enumerate((6000, 15000))]
    n0 = [2000, 9000]
    clouds = [(P, A.Cloud.build(P[:n]).upload()) for P, n in zip(Pfull, n0)]
    torch.cuda.synchronize()
    # per cloud: the list of (n, live mask over the full stream) after v update batches
    states = [[(n, np.concatenate([np.ones(n, np.uint8), np.zeros(P.shape[0] - n, np.uint8)]))]
              for (P, _), n in zip(clouds, n0)]
    rng = np.random.default_rng(12)
    srv = A.Server(pool_queries=1 << 15, nstreams=2, max_wave_requests=16, plain=mode == "plain",
                   lazy_delete=mode == "lazy_delete")
    log = []
    for step in range(60):
        c = int(rng.integers(2))
        P, cl = clouds[c]
        n, live = states[c][-1]
        u = rng.uniform()
        if u < 0.2 and n + 600 <= P.shape[0]:
            cnt = int(rng.integers(1, 600))
            nxt = live.copy()
            nxt[n:n + cnt] = 1
            states[c].append((n + cnt, nxt))
            log.append(("ins", srv.insert(cl, P[n:n + cnt]), c, None, None, None))
        elif u < 0.3:
            alive = np.flatnonzero(live)
            dead = rng.choice(alive, int(rng.integers(1, 100)), replace=False)
            nxt = live.copy()
            nxt[dead] = 0
            states[c].append((n, nxt))
            log.append(("del", srv.delete(cl, dead), c, None, None, None))
        else:
            nq = int(rng.choice([50, 500, 2000]))
            k = int(rng.choice([4, 16, 40]))
            Q = W.uniform_in_box(rng, nq, *W.bbox_expanded(P, 1.1))
            log.append(("knn", srv.submit(cl, torch.from_numpy(Q).cuda(), k), c, Q, k,
                        len(states[c]) - 1))
    res = {t: srv.wait(t, with_seen=True) for _, t, *_ in log}
    srv.close()
    assert any(kind == "ins" for kind, *_ in log)
    ex = 0
    for kind, t, c, Q, k, before in log:
        if kind != "knn":
            continue
        _, _, (_, idx, dist, *_), seen = res[t]
        assert seen == before
        n, live = states[c][seen]
        P = clouds[c][0][:n]
        sel = np.arange(min(100, Q.shape[0]))
        ri, _, rD = oracle.knn_bruteforce(P, Q[sel], k + 1, live=live[:n])
        ex += compare_rows(idx.cpu().numpy()[sel], dist.cpu().numpy()[sel], ri[:, :k],
                           rD[:, :k], rD[:, k], P=P, Q=Q[sel], live=live[:n])
    assert ex <= 2
    for c, (P, cl) in enumerate(clouds):
        n, live = states[c][-1]
        assert cl.n == n and cl.live_count == int(live.sum())


def test_lazy_delete_answers_uncertified_rows_again(env):
    """Deleting the 80 nearest sites of some queries leaves their k + 16 walks on the
    un-updated lists without k unmarked sites; those requests are answered again once the
    deletions in their view are applied.  Requests submitted before each deletion still see
    its sites, and the ones after it do not."""
    torch, oracle, A, W = env
    P = W.random_cloud(30000, seed=95, shape="torus").by_rank
    cl = A.Cloud.build(P).upload()
    torch.cuda.synchronize()
    rng = np.random.default_rng(96)
    centres = P[rng.choice(P.shape[0], 6, replace=False)]
    masks = [np.ones(P.shape[0], np.uint8)]
    srv = A.Server(pool_queries=1 << 15, nstreams=2, max_wave_requests=16, lazy_delete=True)
    log = []
    for i, c0 in enumerate(centres):
        live = masks[-1]
        ri, _, rD = oracle.knn_bruteforce(P, c0[None, :], 80, live=live)
        # queries well inside the disc of the 80 sites about to be deleted
        sd = float(np.sqrt(rD[0, -1])) / 20
        Q = (c0[None, :] + rng.normal(0, sd, (300, 3))).astype(np.float32)
        log.append(("knn", srv.submit(cl, torch.from_numpy(Q).cuda(), 16), Q, len(masks) - 1))
        dead = ri[0]
        nxt = live.copy()
        nxt[dead] = 0
        masks.append(nxt)
        log.append(("del", srv.delete(cl, dead), None, None))
        log.append(("knn", srv.submit(cl, torch.from_numpy(Q).cuda(), 16), Q, len(masks) - 1))
    res = {t: srv.wait(t, with_seen=True) for _, t, *_ in log}
    srv.close()
    ex = 0
    for kind, t, Q, before in log:
        if kind != "knn":
            continue
        _, _, (_, idx, dist, *_), seen = res[t]
        assert seen == before
        ri, _, rD = oracle.knn_bruteforce(P, Q, 16, live=masks[seen])
        ex += compare_rows(idx.cpu().numpy(), dist.cpu().numpy(), ri, rD, P=P, Q=Q,
                           live=masks[seen])
    assert ex <= 2
    assert cl.live_count == int(masks[-1].sum())


def test_lazy_delete_errors(env):
    torch, oracle, A, W = env
    from paper_2605_02224_amd._lib import MknnError, ENOTFOUND, EINVAL
    for kw in ({"plain": True}, {"bind_at_admission": True}):
        with pytest.raises(MknnError) as e:
            A.Server(pool_queries=1000, lazy_delete=True, **kw)
        assert e.value.status == EINVAL
    (P, cl), = _clouds(env, 1, seed=97, nmax=3000)
    n = P.shape[0]
    srv = A.Server(pool_queries=1 << 14, nstreams=2, max_wave_requests=4, lazy_delete=True)
    bad = [srv.delete(cl, [n]), srv.delete(cl, [3, 3]), srv.delete(cl, np.arange(n))]
    good = srv.delete(cl, [5])
    again = srv.delete(cl, [5])                   # already deleted (marked) before it
    q = torch.from_numpy(P[:8]).cuda()
    t = srv.submit(cl, q, 2)
    for b, st in zip(bad, (ENOTFOUND, ENOTFOUND, EINVAL)):
        with pytest.raises(MknnError) as e:
            srv.wait(b)
        assert e.value.status == st
    srv.wait(good)
    with pytest.raises(MknnError) as e:
        srv.wait(again)
    assert e.value.status == ENOTFOUND
    _, _, (_, idx, dist, *_), seen = srv.wait(t, with_seen=True)
    assert seen == 1                              # the one good deletion
    idx = idx.cpu().numpy()
    assert idx[:, 0].tolist() == [0, 1, 2, 3, 4, int(idx[5, 0]), 6, 7]
    assert idx[5, 0] != 5
    srv.close()
    # a cloud with deletions pending from the plain call cannot be served lazily
    cl.delete_lazy([7])
    srv = A.Server(pool_queries=1 << 14, nstreams=2, max_wave_requests=4, lazy_delete=True)
    with pytest.raises(MknnError) as e:
        srv.submit(cl, q, 2)
    assert e.value.status == EINVAL
    srv.close()
    cl.flush()
