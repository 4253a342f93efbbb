"""Reference local plane fit on k-NN rows -- TEST INFRASTRUCTURE ONLY.

The paper motivates k-NN with local neighbourhood statistics (normal estimation, surface
fitting; the limitations of 1-NN search listed in Sec. 3) and uses exactly that in its scan
convergence study (Sec. 5.3.1): the k = 20 nearest neighbours of a probe within the first
m points are fitted with a plane by PCA, and the fitting residual decides convergence.
The paper does not define the residual; the readings used here (also in the design notes)
are:
  * the plane passes through the centroid c of the neighbours and is normal to the
    eigenvector of the smallest eigenvalue lambda_0 of the covariance
    C = (1/k') sum (p - c)(p - c)^T over the k' neighbours found (k' <= k);
  * the residual is the RMS distance of the neighbours to that plane, sqrt(lambda_0);
  * the surface variation lambda_0 / (lambda_0 + lambda_1 + lambda_2) is reported too
    (0 when all three vanish);
  * the normal's sign: its largest-magnitude component is positive (the first of equal
    magnitudes);
  * with fewer than three neighbours the plane is undefined: normal, residual and
    variation are NaN (the centroid is still given when there is at least one).
Everything in float64; the eigen decomposition is LAPACK's (numpy.linalg.eigh).
"""
from __future__ import annotations

import numpy as np

NAN = float("nan")


def plane_fit(points: np.ndarray):
    """points: [k', 3] -> (centroid[3], normal[3], rms, variation), float64."""
    p = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    if p.shape[0] == 0:
        return np.full(3, NAN), np.full(3, NAN), NAN, NAN
    c = p.mean(axis=0)
    if p.shape[0] < 3:
        return c, np.full(3, NAN), NAN, NAN
    X = p - c
    C = X.T @ X / p.shape[0]
    w, V = np.linalg.eigh(C)          # ascending eigenvalues
    n = V[:, 0].copy()
    i = int(np.argmax(np.abs(n)))
    if n[i] < 0:
        n = -n
    lam0 = max(float(w[0]), 0.0)
    tot = float(max(w[0], 0.0) + max(w[1], 0.0) + max(w[2], 0.0))
    return c, n, float(np.sqrt(lam0)), (lam0 / tot if tot > 0 else 0.0)


def plane_fit_rows(points_by_rank: np.ndarray, idx: np.ndarray):
    """Plane of every k-NN row (ranks, -1 = padding) -> float64 [nq, 8]:
    centroid xyz, normal xyz, rms residual, surface variation."""
    P = np.asarray(points_by_rank, dtype=np.float64)
    out = np.empty((idx.shape[0], 8))
    for q in range(idx.shape[0]):
        row = idx[q]
        c, n, rms, var = plane_fit(P[row[row >= 0]])
        out[q, 0:3] = c
        out[q, 3:6] = n
        out[q, 6] = rms
        out[q, 7] = var
    return out
