"""Brute-force successor lists -- TEST INFRASTRUCTURE ONLY (never used by the product path).

Definition (Sec. 3, successor lists; Fig. 2 caption): for points ordered by birth,
p_0, p_1, ... (0-based ranks), the list L_i holds the younger ranks j > i whose arrival cut
away part of the Voronoi cell p_i had among the points born before p_j.  A cell loses a part
of positive volume to p_j exactly when, in the Voronoi diagram of {p_0..p_j}, the cells of
p_i and p_j meet in a facet of positive area -- the test implemented below.  Ranks are
appended in birth order, so each list ascends.

Exact test for one pair: the shared facet lies in the bisector plane of p_i, p_j, and it has
positive area iff some point x of that plane is strictly closer to p_i (equivalently p_j)
than to every other point of the prefix.  Each other point p_k contributes one strict
linear inequality 2 x.(p_k - p_i) < |p_k|^2 - |p_i|^2 on the plane.  Feasibility of a
system of strict linear inequalities in the plane's two free coordinates is decided by
Fourier-Motzkin elimination, which is exact for strict inequalities.  All arithmetic is on
Python integers: float32 coordinates are dyadic rationals, scaled to integers by a common
power of two (a uniform scaling changes no adjacency).

Cost is O(n^4) overall: meant for tiny clouds (tens of points).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence

import numpy as np


def to_integer_coords(points: np.ndarray) -> List[tuple]:
    """Exact integer images of float32 (or float64) coordinates under one 2^s scaling."""
    fr = [[Fraction(float(v)) for v in row] for row in np.asarray(points, dtype=np.float64)]
    den = 1
    for row in fr:
        for v in row:
            den = max(den, v.denominator)
    return [tuple(int(v * den) for v in row) for row in fr]


def _strict_system_feasible(cons) -> bool:
    """cons: list of (alpha, beta, gamma) meaning alpha*s + beta*t < gamma (integers).

    Eliminate s, then decide the one-variable system in t."""
    upper, lower, rest = [], [], []
    for a, b, g in cons:
        if a > 0:
            upper.append((a, b, g))
        elif a < 0:
            lower.append((a, b, g))
        else:
            rest.append((b, g))
    # a1 > 0: s < (g1 - b1 t)/a1 ; a2 < 0: s > (g2 - b2 t)/a2.  Need lower < upper:
    # multiply the first by -a2 > 0, the second by a1 > 0 and add.
    for a1, b1, g1 in upper:
        for a2, b2, g2 in lower:
            rest.append((-a2 * b1 + a1 * b2, -a2 * g1 + a1 * g2))
    lo = None   # t > lo (as Fraction)
    hi = None   # t < hi
    for b, g in rest:
        if b == 0:
            if not (0 < g):
                return False
        elif b > 0:
            v = Fraction(g, b)
            hi = v if hi is None or v < hi else hi
        else:
            v = Fraction(g, b)
            lo = v if lo is None or v > lo else lo
    return lo is None or hi is None or lo < hi


def strongly_adjacent(P: Sequence[tuple], i: int, j: int, members: Sequence[int]) -> bool:
    """True iff the Voronoi cells of P[i] and P[j] within the set `members` (which contains
    i and j) share a facet of positive area.  P holds exact integer coordinates."""
    pi, pj = P[i], P[j]
    n = [pj[d] - pi[d] for d in range(3)]
    # choose a coordinate axis with n[a] != 0 to solve the plane equation for x[a]
    a = max(range(3), key=lambda d: abs(n[d]))
    if n[a] == 0:
        raise ValueError("duplicate points")
    b, c = [d for d in range(3) if d != a]
    sgn = 1 if n[a] > 0 else -1
    na_abs = abs(n[a])
    pi2 = sum(v * v for v in pi)
    h = sum(v * v for v in pj) - pi2          # plane: 2 n.x = h
    cons = []
    for k in members:
        if k == i or k == j:
            continue
        pk = P[k]
        w = [pk[d] - pi[d] for d in range(3)]
        hk = sum(v * v for v in pk) - pi2     # constraint: 2 w.x < hk
        # substitute 2 n_a x_a = h - 2 n_b s - 2 n_c t, multiply by |n_a|
        alpha = sgn * 2 * (n[a] * w[b] - w[a] * n[b])
        beta = sgn * 2 * (n[a] * w[c] - w[a] * n[c])
        gamma = na_abs * hk - sgn * w[a] * h
        cons.append((alpha, beta, gamma))
    return _strict_system_feasible(cons)


def successor_lists(points_by_rank: np.ndarray) -> List[List[int]]:
    """L[i] = ascending ranks j > i with p_i, p_j facet-adjacent in Vor({p_0..p_j})."""
    P = to_integer_coords(points_by_rank)
    nn = len(P)
    L: List[List[int]] = [[] for _ in range(nn)]
    for j in range(1, nn):
        members = list(range(j + 1))
        for i in range(j):
            if strongly_adjacent(P, i, j, members):
                L[i].append(j)
    return L


def weakly_adjacent_pairs_at_insertion(points_by_rank: np.ndarray) -> List[set]:
    """For degenerate inputs: W[j] = {i < j : some closed ball through p_i and p_j contains
    no point of {p_0..p_j} in its interior}.  Facet adjacency implies this; in general
    position the two coincide.  A ball through p_i, p_j is empty iff its centre x on the
    bisector plane has |x-p_i| <= |x-p_k| for all k, i.e. the non-strict version of the
    system above; it is decided here by exact rational vertex enumeration of the 2-D
    polygon (feasible iff the closed polygon is non-empty)."""
    P = to_integer_coords(points_by_rank)
    nn = len(P)
    W = [set() for _ in range(nn)]
    for j in range(1, nn):
        for i in range(j):
            if _closed_bisector_region_nonempty(P, i, j, range(j + 1)):
                W[j].add(i)
    return W


def _closed_bisector_region_nonempty(P, i, j, members) -> bool:
    pi, pj = P[i], P[j]
    n = [pj[d] - pi[d] for d in range(3)]
    a = max(range(3), key=lambda d: abs(n[d]))
    b, c = [d for d in range(3) if d != a]
    sgn = 1 if n[a] > 0 else -1
    na_abs = abs(n[a])
    pi2 = sum(v * v for v in pi)
    h = sum(v * v for v in pj) - pi2
    cons = []
    for k in members:
        if k == i or k == j:
            continue
        pk = P[k]
        w = [pk[d] - pi[d] for d in range(3)]
        hk = sum(v * v for v in pk) - pi2
        cons.append((sgn * 2 * (n[a] * w[b] - w[a] * n[b]),
                     sgn * 2 * (n[a] * w[c] - w[a] * n[c]),
                     na_abs * hk - sgn * w[a] * h))
    # non-strict Fourier-Motzkin: alpha s + beta t <= gamma
    upper, lower, rest = [], [], []
    for a1, b1, g1 in cons:
        if a1 > 0:
            upper.append((a1, b1, g1))
        elif a1 < 0:
            lower.append((a1, b1, g1))
        else:
            rest.append((b1, g1))
    for a1, b1, g1 in upper:
        for a2, b2, g2 in lower:
            rest.append((-a2 * b1 + a1 * b2, -a2 * g1 + a1 * g2))
    lo = hi = None
    for bb, g in rest:
        if bb == 0:
            if g < 0:
                return False
        elif bb > 0:
            v = Fraction(g, bb)
            hi = v if hi is None or v < hi else hi
        else:
            v = Fraction(g, bb)
            lo = v if lo is None or v > lo else lo
    return lo is None or hi is None or lo <= hi
