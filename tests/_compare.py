"""Comparison of GPU k-NN rows with the oracle's, under the stated near-tie rule.

Rule: neighbour index lists must equal the oracle's except at near-ties.  A position may
differ only when the oracle distances there are tied to within 1e-6 relative with a
neighbouring position (an order swap or the k-th/(k+1)-th set boundary); such positions
are counted.  Returned float32 distances must be within 1e-5 relative of the oracle's
float64 distances, and exactly 0 where the oracle distance is 0.
"""
from __future__ import annotations

import numpy as np

NEAR_TIE_REL = 1e-6
DIST_REL = 1e-5


def compare_rows(gpu_idx, gpu_dist, ref_idx, ref_D, ref_D_next=None):
    """gpu_idx/gpu_dist: [nq,k]; ref_idx/ref_D: oracle [nq,k] (ranks, float64 D).

    ref_D_next: optional oracle D of the (k+1)-th neighbour per row, to excuse a boundary
    near-tie.  Returns the number of excused near-tie positions; raises AssertionError on
    any other difference."""
    gi = np.asarray(gpu_idx)
    gd = np.asarray(gpu_dist, dtype=np.float64)
    ri = np.asarray(ref_idx)
    rd = np.sqrt(np.asarray(ref_D, dtype=np.float64))
    assert gi.shape == ri.shape, (gi.shape, ri.shape)
    pad = ri < 0
    assert (gi[pad] == -1).all(), "padding mismatch"
    assert np.isinf(gd[pad]).all(), "padding distance must be +inf"
    live = ~pad
    zero = live & (rd == 0)
    assert (gd[zero] == 0).all(), "zero distances must be exact"
    nz = live & (rd > 0)
    rel = np.abs(gd[nz] - rd[nz]) / rd[nz]
    assert rel.size == 0 or rel.max() <= DIST_REL, f"distance rel err {rel.max():.3e}"
    bad = np.argwhere(gi != ri)
    excused = 0
    for t, j in bad:
        d = rd[t]
        ok = False
        if j > 0 and abs(d[j] - d[j - 1]) <= NEAR_TIE_REL * max(d[j], 1e-300):
            ok = True
        if j + 1 < d.shape[0] and abs(d[j + 1] - d[j]) <= NEAR_TIE_REL * max(d[j], 1e-300):
            ok = True
        if not ok and j == d.shape[0] - 1 and ref_D_next is not None:
            dn = np.sqrt(ref_D_next[t])
            ok = abs(dn - d[j]) <= NEAR_TIE_REL * max(d[j], 1e-300)
        assert ok, f"row {t} pos {j}: gpu {gi[t].tolist()} oracle {ri[t].tolist()}"
        excused += 1
    return excused
