"""Pins of the reference plane fit (oracle/planefit.py) to facts that do not depend on it:
points on a known plane, the residual as a directly summed RMS distance, the normal as the
minimiser of the squared residual, rigid-motion invariance and a configuration with known
covariance."""
import numpy as np
import pytest

from oracle import planefit as PF


def _rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    return q * np.sign(np.diag(r))


def test_points_on_a_known_plane():
    # z = 0.5 x - 0.25 y + 2, on a grid of exactly representable values
    g = np.arange(-3, 4, dtype=np.float64) / 4
    x, y = np.meshgrid(g, g)
    P = np.stack([x.ravel(), y.ravel(), 0.5 * x.ravel() - 0.25 * y.ravel() + 2.0], axis=1)
    c, n, rms, var = PF.plane_fit(P)
    want = np.array([-0.5, 0.25, 1.0]) / np.linalg.norm([-0.5, 0.25, 1.0])
    assert np.allclose(n, want, atol=1e-12)          # largest component (z) positive
    assert np.allclose(c, [0.0, 0.0, 2.0], atol=1e-15)
    assert rms < 1e-7 and var < 1e-14


def test_known_covariance():
    # +-a e_x, +-b e_y, +-c e_z: covariance diag(a^2, b^2, c^2) / 3
    a, b, cc = 3.0, 2.0, 0.5
    P = np.array([[a, 0, 0], [-a, 0, 0], [0, b, 0], [0, -b, 0], [0, 0, cc], [0, 0, -cc]])
    c, n, rms, var = PF.plane_fit(P)
    assert np.allclose(c, 0) and np.allclose(np.abs(n), [0, 0, 1])
    assert rms == pytest.approx(cc / np.sqrt(3), rel=1e-12)
    assert var == pytest.approx(cc * cc / (a * a + b * b + cc * cc), rel=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_residual_is_rms_distance_and_minimal(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(3, 40))
    P = rng.standard_normal((k, 3)) * [1.0, 0.7, 0.05] @ _rot(rng).T + rng.uniform(-5, 5, 3)
    c, n, rms, var = PF.plane_fit(P)
    assert np.linalg.norm(n) == pytest.approx(1.0, abs=1e-12)
    direct = np.sqrt(np.mean(((P - c) @ n) ** 2))
    assert rms == pytest.approx(direct, rel=1e-9, abs=1e-15)
    # no other unit direction through the centroid fits better
    U = rng.standard_normal((2000, 3))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    others = np.sqrt(np.mean(((P - c) @ U.T) ** 2, axis=0))
    assert (others >= rms * (1 - 1e-12)).all()
    # the centroid is the mean
    assert np.allclose(c, P.mean(axis=0), atol=1e-13)


def test_rigid_motion_moves_the_plane_with_the_points():
    rng = np.random.default_rng(9)
    P = rng.standard_normal((25, 3)) * [2.0, 1.0, 0.1]
    R, t = _rot(rng), rng.uniform(-3, 3, 3)
    c0, n0, r0, v0 = PF.plane_fit(P)
    c1, n1, r1, v1 = PF.plane_fit(P @ R.T + t)
    assert np.allclose(c1, R @ c0 + t, atol=1e-12)
    assert abs(abs(np.dot(n1, R @ n0)) - 1) < 1e-10
    assert r1 == pytest.approx(r0, rel=1e-9) and v1 == pytest.approx(v0, rel=1e-9)


def test_too_few_points_and_padding():
    c, n, rms, var = PF.plane_fit(np.array([[1.0, 2.0, 3.0], [3.0, 2.0, 1.0]]))
    assert np.allclose(c, [2, 2, 2]) and np.isnan(n).all() and np.isnan(rms) and np.isnan(var)
    P = np.random.default_rng(1).standard_normal((10, 3))
    out = PF.plane_fit_rows(P, np.array([[0, 1, 2, 3, -1], [4, -1, -1, -1, -1]]))
    assert np.allclose(out[0, :3], P[:4].mean(axis=0)) and not np.isnan(out[0, 3:]).any()
    assert np.allclose(out[1, :3], P[4]) and np.isnan(out[1, 3:]).all()
