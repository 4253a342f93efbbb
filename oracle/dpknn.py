"""Reference walk of the paper's query algorithms -- TEST INFRASTRUCTURE ONLY.

Takes the steps of Alg. 1 (transition-site collection during the 1-NN descent) and Alg. 2
(k-NN by expanding the successor lists of the confirmed neighbours) in the paper's order, on
successor lists given as Python lists.  It exists to check, on the CPU, that a successor
table is sufficient for exact k-NN (Theorem 1), and to count the work the method does per
query: entries examined E(q) and lists opened Lambda(q).

Readings of the paper used here (each is also listed in the design notes):
  * distances are compared through the float64 key (D, rank) with D rounded exactly as in the
    brute-force oracle; "closer" in Alg. 1 is the strict key comparison, so the older site
    wins an exact tie;
  * after a jump in Alg. 1 the scan restarts at the first entry of the new list (all of its
    entries are younger than the site just reached);
  * N has capacity k and is kept sorted by key; Alg. 2's "not in N" is membership in the
    current N;
  * a prefix bound m skips every rank >= m (Sec. 4.2, prefix-subset queries); since lists
    are ascending, a scan stops at the first such rank;
  * deleted ranks never appear in the lists, and the descent starts from the oldest live
    rank (the head).
Pure Python: meant for small inputs.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np


def _D(q, p) -> float:
    dx = float(q[0]) - float(p[0])
    dy = float(q[1]) - float(p[1])
    dz = float(q[2]) - float(p[2])
    return (dx * dx + dy * dy) + dz * dz


class _Candidates:
    """Sorted candidate list N of capacity k, ordered by (D, rank)."""

    def __init__(self, k: int):
        self.k = k
        self.items: List[Tuple[float, int]] = []

    def insert(self, d: float, r: int) -> None:
        key = (d, r)
        if key in self.items:
            return
        if len(self.items) == self.k and not key < self.items[-1]:
            return
        pos = len(self.items)
        while pos > 0 and key < self.items[pos - 1]:
            pos -= 1
        self.items.insert(pos, key)
        if len(self.items) > self.k:
            self.items.pop()


def dp_knn(points_by_rank: np.ndarray, lists: Sequence[Sequence[int]], q, k: int,
           m: Optional[int] = None, head: int = 0, count: bool = False):
    """k nearest ranks of q within ranks < m, as [(D, rank), ...] ascending.

    With count=True also returns (E, Lambda): entries examined and lists opened, where the
    final list of the descent, which Alg. 2's first iteration scans again, is counted once.
    """
    P = points_by_rank
    n = len(lists)
    if m is None:
        m = n
    N = _Candidates(k)
    E = 0
    lam = 0
    if head >= m:
        return (N.items, (0, 0)) if count else N.items
    # ---- Alg. 1: descend from the head, collecting transition sites into N
    cur = head
    dcur = _D(q, P[cur])
    N.insert(dcur, cur)
    lam += 1
    pos = 0
    lst = lists[cur]
    while pos < len(lst):
        r = lst[pos]
        if r >= m:
            break
        E += 1
        d = _D(q, P[r])
        if (d, r) < (dcur, cur):
            cur, dcur = r, d
            N.insert(d, r)
            lst = lists[cur]
            pos = 0
            lam += 1
            continue
        pos += 1
    nn = cur
    # ---- Alg. 2: for i = 1..k-1 expand the list of the i-th confirmed neighbour
    for i in range(k - 1):
        if i >= len(N.items):
            break
        p = N.items[i][1]
        if p != nn:
            lam += 1
        for r in lists[p]:
            if r >= m:
                break
            if p != nn:
                E += 1
            N.insert(_D(q, P[r]), r)
    return (N.items, (E, lam)) if count else N.items


def dp_knn_batch(points_by_rank: np.ndarray, lists, queries: np.ndarray, k: int,
                 m: Optional[int] = None, head: int = 0):
    """Rows of (ranks int32 [nq,k] padded -1, D float64 [nq,k] padded +inf, E, Lambda)."""
    nq = queries.shape[0]
    idx = np.full((nq, k), -1, dtype=np.int32)
    D = np.full((nq, k), np.inf)
    E = np.zeros(nq, dtype=np.int64)
    lam = np.zeros(nq, dtype=np.int64)
    for t in range(nq):
        items, (e, l) = dp_knn(points_by_rank, lists, queries[t], k, m, head, count=True)
        for j, (d, r) in enumerate(items):
            idx[t, j] = r
            D[t, j] = d
        E[t] = e
        lam[t] = l
    return idx, D, E, lam
