"""Pins for the brute-force k-NN oracle against facts it does not compute itself."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _exact_D(q, p):
    return sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(q, p))


def test_hand_worked_example(oracle_lib):
    g = json.load(open(os.path.join(HERE, "golden", "knn_hand_example.json")))
    P = np.array(g["points_by_rank"], dtype=np.float32)
    for c in g["cases"]:
        q = np.array([c["q"]], dtype=np.float32)
        idx, dist, D = oracle_lib.knn_bruteforce(P, q, c["k"], c["m"])
        assert idx[0].tolist() == c["ranks"], c
        want = [math.inf if v == "inf" else float(v) for v in c["D"]]
        assert D[0].tolist() == want
        assert np.allclose(dist[0], np.sqrt(np.array(want)), rtol=1e-7)


def test_exhaustive_lexicographic_minimum(oracle_lib):
    """Tiny clouds on a coarse grid (many exact ties): for every query, k and prefix m, the
    answer's key sequence is the lexicographic minimum over all k-subsets of the prefix,
    with keys (exact rational D, rank)."""
    rng = np.random.default_rng(11)
    for trial in range(6):
        n = int(rng.integers(3, 9))
        P = (rng.integers(-6, 7, (n, 3)) / 4.0).astype(np.float32)
        P = np.unique(P, axis=0)
        rng.shuffle(P)
        n = P.shape[0]
        Q = (rng.integers(-8, 9, (4, 3)) / 4.0).astype(np.float32)
        for m in range(1, n + 1):
            for k in range(1, n + 2):
                idx, dist, D = oracle_lib.knn_bruteforce(P, Q, k, m)
                for t in range(Q.shape[0]):
                    keys = sorted((_exact_D(Q[t], P[r]), r) for r in range(m))
                    best = None
                    kk = min(k, m)
                    for sub in itertools.combinations(range(m), kk):
                        seq = sorted((_exact_D(Q[t], P[r]), r) for r in sub)
                        if best is None or seq < best:
                            best = seq
                    assert idx[t, :kk].tolist() == [r for _, r in best]
                    assert [Fraction(v) for v in D[t, :kk]] == [d for d, _ in best]
                    assert (idx[t, kk:] == -1).all() and np.isinf(dist[t, kk:]).all()
                    assert keys[:kk] == best


def test_matches_kdtree_on_random_surface(oracle_lib):
    """scipy's kd-tree (an independent exact k-NN) agrees on a 20k-point torus sample,
    apart from near-ties at the boundary."""
    from scipy.spatial import cKDTree
    from paper_2605_02224_amd import workloads as W
    c = W.random_cloud(20000, seed=3, shape="torus")
    P = c.by_rank
    rng = np.random.default_rng(5)
    lo, hi = W.bbox_expanded(P, 1.1)
    Q = W.uniform_in_box(rng, 3000, lo, hi)
    k = 16
    idx, dist, D = oracle_lib.knn_bruteforce(P, Q, k)
    dd, ii = cKDTree(P.astype(np.float64)).query(Q.astype(np.float64), k=k)
    mism = 0
    for t in range(Q.shape[0]):
        if idx[t].tolist() != ii[t].tolist():
            # only tolerated where the kd-tree's own distances tie to 1e-12
            a = dd[t]
            swaps = [j for j in range(k) if idx[t, j] != ii[t, j]]
            for j in swaps:
                assert abs(math.sqrt(D[t, j]) - a[j]) <= 1e-9 * max(a[j], 1e-30)
            mism += 1
        assert np.allclose(np.sqrt(D[t]), dd[t], rtol=1e-12, atol=0)
    assert mism <= 3


def test_argmin_special_case(oracle_lib):
    """k=1 is the argmin of the squared distances (first minimum = smallest rank)."""
    rng = np.random.default_rng(2)
    P = rng.standard_normal((500, 3)).astype(np.float32)
    Q = rng.standard_normal((200, 3)).astype(np.float32)
    idx, dist, D = oracle_lib.knn_bruteforce(P, Q, 1)
    d2 = ((Q[:, None, :].astype(np.float64) - P[None, :, :].astype(np.float64)) ** 2).sum(-1)
    assert (idx[:, 0] == np.argmin(d2, axis=1)).all()


def test_full_sort_special_case(oracle_lib):
    """k >= m returns the whole prefix, stably sorted by distance."""
    rng = np.random.default_rng(3)
    P = (rng.integers(-3, 4, (40, 3))).astype(np.float32)
    P = np.unique(P, axis=0)
    Q = (rng.integers(-3, 4, (30, 3)) + 0.5).astype(np.float32)
    m = 25
    idx, dist, D = oracle_lib.knn_bruteforce(P, Q, 30, m)
    for t in range(Q.shape[0]):
        d = [float(_exact_D(Q[t], P[r])) for r in range(m)]
        want = sorted(range(m), key=lambda r: (d[r], r))
        assert idx[t, :m].tolist() == want
        assert (idx[t, m:] == -1).all()


def test_prefix_live_mask_and_per_query(oracle_lib):
    rng = np.random.default_rng(4)
    P = rng.standard_normal((300, 3)).astype(np.float32)
    Q = rng.standard_normal((50, 3)).astype(np.float32)
    live = np.ones(300, np.uint8)
    dead = rng.choice(300, 40, replace=False)
    live[dead] = 0
    idx, _, _ = oracle_lib.knn_bruteforce(P, Q, 8, 200, live=live)
    assert not np.isin(idx, dead).any()
    assert (idx < 200).all()
    # a dead rank is equivalent to removing its row (relative order kept)
    keep = np.flatnonzero(live)
    idx2, _, _ = oracle_lib.knn_bruteforce(P[keep], Q, 8, int((keep < 200).sum()))
    assert (keep[idx2] == idx).all()
    # per-query k and m with ragged rows agree with scalar calls
    kq = rng.choice([1, 3, 8], 50).astype(np.int32)
    mq = rng.integers(1, 301, 50).astype(np.int32)
    fi, fd, fD, off = oracle_lib.knn_bruteforce(P, Q, k_per_query=kq, m_per_query=mq)
    for t in range(50):
        a, _, _ = oracle_lib.knn_bruteforce(P, Q[t:t + 1], int(kq[t]), int(mq[t]))
        assert fi[off[t]:off[t + 1]].tolist() == a[0].tolist()


def test_zero_distance_and_empty_batch(oracle_lib):
    P = np.array([[0, 0, 0], [1, 2, 3], [-1, 0.5, 2]], np.float32)
    idx, dist, D = oracle_lib.knn_bruteforce(P, P[1:2], 2)
    assert idx[0].tolist() == [1, 2] and dist[0, 0] == 0.0 and D[0, 0] == 0.0
    idx, dist, D = oracle_lib.knn_bruteforce(P, np.zeros((0, 3), np.float32), 2)
    assert idx.shape == (0, 2)


def test_work_counts_hand_trace():
    """The work counts of the reference walk (entries examined E, lists opened Lambda, the
    inputs of the algorithmic-byte figure) equal a hand-counted trace of Alg. 1 + Alg. 2."""
    from oracle import dpknn
    g = json.load(open(os.path.join(HERE, "golden", "dpknn_work_counts.json")))
    P = np.array(g["points_by_rank"], dtype=np.float32)
    for c in g["cases"]:
        items, (E, lam) = dpknn.dp_knn(P, g["lists"], np.array(c["q"], np.float32), c["k"],
                                       c["m"], count=True)
        assert [r for _, r in items] == c["ranks"], c
        assert (E, lam) == (c["E"], c["Lambda"]), c
