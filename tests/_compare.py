"""Comparison of GPU k-NN rows with the oracle's, under the stated near-tie rule.

Rule: neighbour index lists must equal the oracle's except at near-ties.  Every GPU row is
first checked on its own:

  * padding (-1, +inf) sits exactly where the oracle pads;
  * every returned rank is a point of the query's set: 0 <= rank < m, live, no rank twice;
  * every returned distance is the distance of the returned rank: its squared distance D is
    recomputed here in float64 from P and the query, by the same formula as the oracle
    (((qx-px)^2 + (qy-py)^2) + (qz-pz)^2, every operation rounded, no fused multiply-add),
    and the float32 distance must be within 1e-5 relative of sqrt(D) (exactly 0 where
    D = 0);
  * the row is ordered by (D, rank).

Then position j may hold a rank other than the oracle's only when that rank's recomputed
distance ties the oracle's distance at j within 1e-6 relative.  Since the oracle row is the
exact k-NN, such a rank either sits elsewhere in the oracle row (an order swap between
tied positions) or lies outside it, at or beyond the oracle's k-th distance (a near-tie at
the set boundary); either way it is a genuine near-tie.  Such positions are counted and the
count is returned; every other difference raises AssertionError.
"""
from __future__ import annotations

import numpy as np

NEAR_TIE_REL = 1e-6
DIST_REL = 1e-5


def recompute_D(P, Q, idx):
    """Float64 squared distances of ranks idx [nq, k] (-1 = none) from queries Q [nq, 3]."""
    P = np.asarray(P, dtype=np.float32)
    Q = np.asarray(Q, dtype=np.float32).reshape(-1, 3)
    idx = np.asarray(idx)
    safe = np.where(idx >= 0, idx, 0)
    p = P[safe].astype(np.float64)                     # [nq, k, 3]
    q = Q.astype(np.float64)[:, None, :]
    d = q - p
    D = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    return np.where(idx >= 0, D, np.inf)


def compare_rows(gpu_idx, gpu_dist, ref_idx, ref_D, ref_D_next=None, *, P, Q, m=None,
                 live=None):
    """gpu_idx/gpu_dist: [nq,k]; ref_idx/ref_D: oracle [nq,k] (ranks, float64 D).

    P: the cloud by rank (float32 [n,3]); Q: the queries of these rows (float32 [nq,3]);
    m: the prefix (scalar, or int array [nq]; None = n); live: bool [n] or None.
    ref_D_next (optional) is unused by the rule but kept for callers that have it.
    Returns the number of excused near-tie positions."""
    gi = np.asarray(gpu_idx).astype(np.int64)
    gd = np.asarray(gpu_dist, dtype=np.float64)
    ri = np.asarray(ref_idx).astype(np.int64)
    rD = np.asarray(ref_D, dtype=np.float64)
    assert gi.shape == ri.shape == gd.shape == rD.shape, (gi.shape, ri.shape)
    if gi.size == 0:
        return 0
    nq, k = gi.shape
    Qa = np.asarray(Q, dtype=np.float32).reshape(-1, 3)
    assert Qa.shape[0] == nq, (Qa.shape, nq)
    n = np.asarray(P).shape[0]
    mm = np.full(nq, n, np.int64) if m is None else np.broadcast_to(
        np.minimum(np.asarray(m, np.int64), n), (nq,))

    # padding exactly where the oracle pads
    pad = ri < 0
    assert (gi[pad] == -1).all(), "padding mismatch: the GPU returned a rank the oracle has not"
    assert (gi[~pad] >= 0).all(), "padding mismatch: the GPU padded where the oracle has a rank"
    assert np.isinf(gd[pad]).all(), "padding distance must be +inf"
    has = ~pad

    # every returned rank lies in the query's set, once
    assert (gi[has] < mm[:, None].repeat(k, 1)[has]).all(), "rank outside the prefix"
    if live is not None:
        lv = np.asarray(live, bool)
        assert lv[gi[has]].all(), "a deleted rank was returned"
    srt = np.sort(np.where(has, gi, -1 - np.arange(k)[None, :]), axis=1)
    assert not (srt[:, 1:] == srt[:, :-1]).any(), "a rank appears twice in a row"

    # every returned distance belongs to the returned rank
    gD = recompute_D(P, Qa, np.where(has, gi, -1))
    gdist = np.sqrt(gD)
    zero = has & (gD == 0)
    assert (gd[zero] == 0).all(), "zero distances must be exact"
    nz = has & (gD > 0)
    rel = np.abs(gd[nz] - gdist[nz]) / gdist[nz]
    assert rel.size == 0 or rel.max() <= DIST_REL, f"distance rel err {rel.max():.3e}"

    # rows ordered by (D, rank)
    if k > 1:
        a, b = gD[:, :-1], gD[:, 1:]
        ra, rb = gi[:, :-1], gi[:, 1:]
        both = has[:, :-1] & has[:, 1:]
        ordered = (a < b) | ((a == b) & (ra < rb))
        assert (ordered | ~both).all(), "a row is not ordered by (D, rank)"

    # differing positions: the GPU rank's own distance ties the oracle's there
    bad = has & (gi != ri)
    if not bad.any():
        return 0
    rdist = np.sqrt(rD)
    tie = np.abs(gdist - rdist) <= NEAR_TIE_REL * np.maximum(rdist, 1e-300)
    wrong = bad & ~tie
    if wrong.any():
        t, j = np.argwhere(wrong)[0]
        raise AssertionError(f"row {t} pos {j}: gpu {gi[t].tolist()} oracle {ri[t].tolist()} "
                             f"(gpu D {gD[t, j]!r}, oracle D {rD[t, j]!r})")
    return int(bad.sum())
