"""Pins for the brute-force successor-list oracle and the reference walk of Alg. 1/2."""
import json
import os

import numpy as np
import pytest

from oracle import successors as S
from oracle import dpknn

HERE = os.path.dirname(os.path.abspath(__file__))


def test_hand_examples():
    g = json.load(open(os.path.join(HERE, "golden", "successors_hand_examples.json")))
    for c in g["cases"]:
        P = np.array(c["points_by_rank"], dtype=np.float32)
        L = S.successor_lists(P)
        if "lists" in c:
            assert L == c["lists"], c["name"]
        else:
            last = P.shape[0] - 1
            owners = [i for i in range(last) if last in L[i]]
            assert owners == c["last_rank_in_lists_of"], c["name"]


def _qhull_lists(P):
    """Successor lists from scipy's Delaunay (Qhull) of every prefix: an independent library."""
    from scipy.spatial import Delaunay
    n = P.shape[0]
    L = [[] for _ in range(n)]
    for j in range(1, n):
        if j < 4:
            nb = set(range(j))      # <= 4 affinely independent sites: all pairs adjacent
        else:
            tri = Delaunay(P[: j + 1].astype(np.float64))
            nb = set()
            for s in tri.simplices:
                if j in s:
                    nb.update(int(v) for v in s if v != j)
        for i in sorted(nb):
            L[i].append(j)
    return L


@pytest.mark.parametrize("seed,shape", [(1, "sphere"), (2, "torus"), (3, "ellipsoid")])
def test_matches_qhull_in_general_position(seed, shape):
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(28, seed=seed, shape=shape, noise=1e-2).by_rank
    assert S.successor_lists(P) == _qhull_lists(P)


def test_lists_ascending_and_strong_equals_weak_generic():
    rng = np.random.default_rng(7)
    P = rng.standard_normal((20, 3)).astype(np.float32)
    L = S.successor_lists(P)
    for i, li in enumerate(L):
        assert li == sorted(li) and all(j > i for j in li)
    W = S.weakly_adjacent_pairs_at_insertion(P)
    for j in range(1, 20):
        assert W[j] == {i for i in range(j) if j in L[i]}


def test_degenerate_lattice_strong_subset_of_weak():
    """On a lattice (cospherical and coplanar everywhere) facet adjacency is contained in
    weak (closed empty ball) adjacency, and face-diagonal-only contacts are excluded."""
    g = np.array([[x, y, z] for x in range(2) for y in range(2) for z in range(2)], np.float32)
    order = [0, 7, 3, 5, 6, 1, 2, 4]
    P = g[order]
    L = S.successor_lists(P)
    W = S.weakly_adjacent_pairs_at_insertion(P)
    for j in range(1, 8):
        strong = {i for i in range(j) if j in L[i]}
        assert strong <= W[j]
    # full cube: the last corner's facet neighbours are exactly its 3 cube-edge neighbours
    last = P[-1]
    edge_nb = {i for i in range(7) if np.abs(P[i] - last).sum() == 1}
    assert {i for i in range(7) if 7 in L[i]} == edge_nb


@pytest.mark.parametrize("seed", [4, 5])
def test_theorem1_on_oracle_lists(seed):
    """Theorem 1 + Alg. 1/2: walking the exact lists reproduces brute-force k-NN for every k
    and prefix m (this pins the walker and the lists together)."""
    import oracle
    oracle.build(force=False)
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(26, seed=seed, shape="sphere", noise=5e-2).by_rank
    L = S.successor_lists(P)
    rng = np.random.default_rng(seed)
    Q = rng.uniform(-1.6, 1.6, (40, 3)).astype(np.float32)
    for m in (1, 2, 5, 13, 26):
        for k in (1, 2, 3, 7, 26, 30):
            ref_idx, _, ref_D = oracle.knn_bruteforce(P, Q, k, m)
            idx, D, E, lam = dpknn.dp_knn_batch(P, L, Q, k, m)
            assert (idx == ref_idx).all(), (m, k)
            assert np.array_equal(D, ref_D)


def test_walker_rejects_incomplete_lists():
    """Dropping one needed list entry must break exactness somewhere (the pin has teeth)."""
    import oracle
    oracle.build(force=False)
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(24, seed=9, shape="torus", noise=5e-2).by_rank
    L = S.successor_lists(P)
    rng = np.random.default_rng(1)
    Q = rng.uniform(-1.4, 1.4, (400, 3)).astype(np.float32)
    ref_idx, _, _ = oracle.knn_bruteforce(P, Q, 6)
    broken = 0
    for i in range(len(L)):
        for e in list(L[i]):
            L2 = [list(x) for x in L]
            L2[i].remove(e)
            idx, _, _, _ = dpknn.dp_knn_batch(P, L2, Q, 6)
            broken += int(not (idx == ref_idx).all())
        if broken >= 3:
            break
    assert broken >= 3


@pytest.mark.parametrize("seed", [6, 7])
def test_entries_nearer_than_a_confirmed_neighbour_are_confirmed(seed):
    """The property the query kernels' expansion uses (from Theorem 1): when the list of the
    i-th nearest site (0-based, i < k-1) is scanned, sites 0 .. i are final, so every entry
    of that list below the prefix bound whose key (D, rank) is below site i's key is one of
    sites 0 .. i-1.  Checked against brute force on the exact lists."""
    import oracle
    oracle.build(force=False)
    from paper_2605_02224_amd import workloads as W
    P = W.random_cloud(26, seed=seed, shape="sphere", noise=5e-2).by_rank
    L = S.successor_lists(P)
    rng = np.random.default_rng(seed)
    Q = rng.uniform(-1.6, 1.6, (60, 3)).astype(np.float32)
    checked = 0
    for m in (2, 9, 17, 26):
        ref_idx, _, ref_D = oracle.knn_bruteforce(P, Q, m, m)
        for q in range(Q.shape[0]):
            order = ref_idx[q].tolist()
            key = {r: (ref_D[q][t], r) for t, r in enumerate(order)}
            for i in range(m - 1):
                owner = order[i]
                for c in L[owner]:
                    if c >= m:
                        break
                    if key[c] < key[owner]:
                        assert c in order[:i], (m, q, i, c)
                        checked += 1
    assert checked > 100
