"""Seeded synthetic workloads: manifold-sampled point clouds, insertion orders and queries.

This module only draws random inputs.  It holds none of the k-NN method's arithmetic and
imports nothing from the rest of the package, so both the HIP path and the CPU oracle can
consume exactly the same bytes.

The paper measures volume-to-surface queries against points sampled on manifolds (Sec. 5,
static k-NN experiments: surface models, queries in an enlarged bounding box, k around
10-20, about a million points).  Its models and datasets are not available here, so the
generators below stand in for them with analytic surfaces (sphere, torus, ellipsoid and a
height field) sampled uniformly by area, a seeded random insertion order and volume
queries in the (enlarged) bounding box.

Seeding scheme (fixed, so every consumer regenerates identical inputs):
  * ``root = SeedSequence(seed)``; children = ``root.spawn(8)``; stream ``i`` is
    ``default_rng(children[i])`` with 0 points, 1 order, 2 queries A, 3 queries B,
    4 per-query prefix m, 5 per-query k, 6 shape parameters and sizes, 7 request stream
    and deletions.
  * The small sphere workload draws its points from ``default_rng(seed)`` directly.
  * Everything is generated in float64 and rounded to float32 last; exact float32
    duplicate points are re-drawn.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# stream indices of SeedSequence(seed).spawn(8)
S_POINTS, S_ORDER, S_QA, S_QB, S_M, S_K, S_SHAPE, S_REQ = range(8)

TORUS_R = 1.0
TORUS_r = 0.3


def _streams(seed: int) -> List[np.random.Generator]:
    return [np.random.default_rng(c) for c in np.random.SeedSequence(seed).spawn(8)]


# --------------------------------------------------------------------------------------
# surface samplers (float64 in, float64 out; callers round to float32)
# --------------------------------------------------------------------------------------
def sample_sphere(rng: np.random.Generator, n: int, noise: float = 0.0):
    """Uniform on the unit sphere (normalised Gaussian vectors), optional normal noise."""
    g = rng.standard_normal((n, 3))
    u = g / np.linalg.norm(g, axis=1, keepdims=True)
    if noise > 0.0:
        u = u * (1.0 + noise * rng.standard_normal((n, 1)))
    return u


def sample_torus(rng: np.random.Generator, n: int, noise: float = 0.0,
                 R: float = TORUS_R, r: float = TORUS_r):
    """Uniform by area on the torus (R, r): u uniform, v accepted with prob (R + r cos v)/(R + r).

    Noise is added along the surface normal (cos v cos u, cos v sin u, sin v).
    """
    us, vs = [], []
    have = 0
    while have < n:
        m = int((n - have) * 1.35) + 64
        u = rng.uniform(0.0, 2.0 * math.pi, m)
        v = rng.uniform(0.0, 2.0 * math.pi, m)
        acc = rng.uniform(0.0, 1.0, m) < (R + r * np.cos(v)) / (R + r)
        us.append(u[acc])
        vs.append(v[acc])
        have += int(acc.sum())
    u = np.concatenate(us)[:n]
    v = np.concatenate(vs)[:n]
    ring = R + r * np.cos(v)
    p = np.stack([ring * np.cos(u), ring * np.sin(u), r * np.sin(v)], axis=1)
    if noise > 0.0:
        nrm = np.stack([np.cos(v) * np.cos(u), np.cos(v) * np.sin(u), np.sin(v)], axis=1)
        p = p + noise * rng.standard_normal((n, 1)) * nrm
    return p


def sample_ellipsoid(rng: np.random.Generator, n: int, axes, noise: float = 0.0):
    """Uniform by area on the ellipsoid with semi-axes (a, b, c), by rejection.

    A unit-sphere point u maps to (a u_x, b u_y, c u_z); its area element is proportional to
    sqrt((bc u_x)^2 + (ac u_y)^2 + (ab u_z)^2), so u is accepted with that value divided by
    max(bc, ac, ab).  Noise is added along the ellipsoid's unit normal.
    """
    a, b, c = (float(x) for x in axes)
    w = np.array([b * c, a * c, a * b])
    wmax = float(w.max())
    pts = []
    have = 0
    while have < n:
        m = int((n - have) * 2.5) + 64
        u = sample_sphere(rng, m)
        dens = np.sqrt(((u * w) ** 2).sum(axis=1)) / wmax
        acc = rng.uniform(0.0, 1.0, m) < dens
        pts.append(u[acc])
        have += int(acc.sum())
    u = np.concatenate(pts)[:n]
    p = u * np.array([a, b, c])
    if noise > 0.0:
        nrm = p / np.array([a * a, b * b, c * c])
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        p = p + noise * rng.standard_normal((n, 1)) * nrm
    return p


def sample_heightfield(rng_xy: np.random.Generator, n: int, coef):
    """z = 0.1 * sum_j sin(a_j x + b_j y + c_j) over (x, y) ~ U[0,1]^2, no noise."""
    a, b, c = coef
    xy = rng_xy.uniform(0.0, 1.0, (n, 2))
    z = 0.1 * np.sin(np.outer(xy[:, 0], a) + np.outer(xy[:, 1], b) + c).sum(axis=1)
    return np.concatenate([xy, z[:, None]], axis=1)


def _dedupe_f32(p64: np.ndarray, redraw) -> np.ndarray:
    """Round to float32 and re-draw rows that duplicate an earlier row exactly."""
    p = p64.astype(np.float32)
    for _ in range(100):
        _, first = np.unique(p.view(np.dtype((np.void, 12))).ravel(), return_index=True)
        if first.size == p.shape[0]:
            return np.ascontiguousarray(p)
        dup = np.setdiff1d(np.arange(p.shape[0]), first)
        p[dup] = redraw(dup.size).astype(np.float32)
    raise RuntimeError("could not remove duplicate points")


def bbox_expanded(p: np.ndarray, factor: float = 1.0):
    """Axis-aligned bounding box, each extent scaled by `factor` about its centre."""
    lo = p.min(axis=0).astype(np.float64)
    hi = p.max(axis=0).astype(np.float64)
    c = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo) * factor
    return c - h, c + h


def uniform_in_box(rng: np.random.Generator, nq: int, lo, hi) -> np.ndarray:
    return rng.uniform(lo, hi, (nq, 3)).astype(np.float32)


# --------------------------------------------------------------------------------------
# clouds
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class Cloud:
    """Points as the caller holds them plus the insertion order (rank r -> point order[r])."""
    points: np.ndarray          # float32 [n,3], caller order
    order: np.ndarray           # int32 [n], a permutation
    shape: str = ""

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def by_rank(self) -> np.ndarray:
        """float32 [n,3] with row r = the r-th inserted point (0-based birth rank)."""
        return np.ascontiguousarray(self.points[self.order])


def _shape_cloud(rng_pts, rng_order, rng_shape, n: int, shape: str, noise: float) -> Cloud:
    if shape == "sphere":
        gen = lambda m: sample_sphere(rng_pts, m, noise)
    elif shape == "torus":
        gen = lambda m: sample_torus(rng_pts, m, noise)
    elif shape == "ellipsoid":
        axes = rng_shape.uniform(0.5, 2.0, 3)
        gen = lambda m: sample_ellipsoid(rng_pts, m, axes, noise)
    else:
        raise ValueError(shape)
    p = _dedupe_f32(gen(n), gen)
    order = rng_order.permutation(n).astype(np.int32)
    return Cloud(p, order, shape)


# --------------------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class PlainWorkload:
    name: str
    cloud: Cloud
    queries: np.ndarray                 # float32 [nq,3]
    k: int                              # scalar k (or max k when per-query k is given)
    m: int                              # scalar prefix (n when full)
    k_per_query: Optional[np.ndarray] = None   # int32 [nq]
    m_per_query: Optional[np.ndarray] = None   # int32 [nq]
    queries_b: Optional[np.ndarray] = None      # second query set (on-surface)


def sphere_small(n: int = 10_000, nq: int = 10_000, k: int = 8, seed: int = 0) -> PlainWorkload:
    """n points uniform on the unit sphere (normalised Gaussians, default_rng(seed)),
    seeded random insertion order, nq queries uniform in [-1.5, 1.5]^3, k=8, m=n."""
    st = _streams(seed)
    rng0 = np.random.default_rng(seed)
    gen = lambda m: sample_sphere(rng0, m)
    p = _dedupe_f32(gen(n), gen)
    order = st[S_ORDER].permutation(n).astype(np.int32)
    q = st[S_QA].uniform(-1.5, 1.5, (nq, 3)).astype(np.float32)
    return PlainWorkload("sphere_10k_k8", Cloud(p, order, "sphere"), q, k, n)


def torus_paper_scale(n: int = 1_000_000, nq: int = 1_000_000, k: int = 16, seed: int = 0,
                      noise: float = 1e-3, jitter: float = 1e-2) -> PlainWorkload:
    """n points on the torus R=1, r=0.3 (uniform by area) with normal noise sigma=1e-3,
    random insertion order; query set A: nq uniform in the bounding box expanded by 10%;
    query set B: nq fresh torus samples jittered by N(0, jitter^2 I)."""
    st = _streams(seed)
    gen = lambda m: sample_torus(st[S_POINTS], m, noise)
    p = _dedupe_f32(gen(n), gen)
    order = st[S_ORDER].permutation(n).astype(np.int32)
    lo, hi = bbox_expanded(p, 1.1)
    qa = uniform_in_box(st[S_QA], nq, lo, hi)
    qb = (sample_torus(st[S_QB], nq, 0.0)
          + jitter * st[S_QB].standard_normal((nq, 3))).astype(np.float32)
    return PlainWorkload(f"torus_{n}_k{k}", Cloud(p, order, "torus"), qa, k, n, queries_b=qb)


def heightfield_prefix(n: int = 2_000_000, nq: int = 2_000_000, seed: int = 0,
                       k_choices=(1, 8, 32)) -> PlainWorkload:
    """n points on z = 0.1 sum_{j<8} sin(a_j x + b_j y + c_j), a,b ~ U[1,20], c ~ U[0,2pi],
    (x,y) ~ U[0,1]^2; random order; nq volume queries in the bbox expanded by 10%, each with
    its own prefix m = round(exp(U[ln(n/1000), ln n])) and k drawn from k_choices."""
    st = _streams(seed)
    a = st[S_SHAPE].uniform(1.0, 20.0, 8)
    b = st[S_SHAPE].uniform(1.0, 20.0, 8)
    c = st[S_SHAPE].uniform(0.0, 2.0 * math.pi, 8)
    gen = lambda m: sample_heightfield(st[S_POINTS], m, (a, b, c))
    p = _dedupe_f32(gen(n), gen)
    order = st[S_ORDER].permutation(n).astype(np.int32)
    lo, hi = bbox_expanded(p, 1.1)
    q = uniform_in_box(st[S_QA], nq, lo, hi)
    lo_m = max(1.0, n / 1000.0)
    mq = np.rint(np.exp(st[S_M].uniform(math.log(lo_m), math.log(n), nq)))
    mq = np.clip(mq, 1, n).astype(np.int32)
    kq = st[S_K].choice(np.asarray(k_choices, dtype=np.int32), nq).astype(np.int32)
    return PlainWorkload(f"heightfield_{n}_prefix", Cloud(p, order, "heightfield"), q,
                         int(max(k_choices)), n, k_per_query=kq, m_per_query=mq)


SHAPES = ("sphere", "torus", "ellipsoid")


@dataclasses.dataclass
class BatchedWorkload:
    name: str
    clouds: List[Cloud]
    queries: List[np.ndarray]
    k: int


def many_clouds(num: int = 256, n_lo: int = 1_000, n_hi: int = 200_000, q_per_point: int = 4,
                k: int = 10, noise: float = 1e-3, seed: int = 0) -> BatchedWorkload:
    """`num` independent clouds, sizes log-uniform in [n_lo, n_hi], each on a random shape
    (sphere, torus, ellipsoid with axes U[0.5,2]^3) with normal noise; each cloud has its own
    random order and q_per_point * n_c queries uniform in its bounding box; k=10, m=n_c."""
    st = _streams(seed)
    sizes = np.rint(np.exp(st[S_SHAPE].uniform(math.log(n_lo), math.log(n_hi), num))).astype(int)
    shapes = st[S_SHAPE].integers(0, len(SHAPES), num)
    clouds, queries = [], []
    for i in range(num):
        c = _shape_cloud(st[S_POINTS], st[S_ORDER], st[S_SHAPE], int(sizes[i]),
                         SHAPES[shapes[i]], noise)
        lo, hi = bbox_expanded(c.points, 1.0)
        clouds.append(c)
        queries.append(uniform_in_box(st[S_QA], q_per_point * c.n, lo, hi))
    return BatchedWorkload(f"batched_{num}_clouds_k{k}", clouds, queries, k)


@dataclasses.dataclass
class Request:
    cloud: int
    queries: np.ndarray
    k: int
    m: int


@dataclasses.dataclass
class ServingWorkload:
    name: str
    clouds: List[Cloud]
    rng_requests: np.random.Generator
    k_choices: tuple = (4, 16, 64)
    max_nq: int = 65536

    def request(self) -> Request:
        """One request: cloud ~ U{0..C-1}, nq = round(exp(U[0, ln max_nq])), k ~ U(k_choices),
        m ~ U{ceil(n/10)..n}, queries uniform in the cloud's bounding box."""
        rng = self.rng_requests
        ci = int(rng.integers(0, len(self.clouds)))
        c = self.clouds[ci]
        nq = int(np.rint(np.exp(rng.uniform(0.0, math.log(self.max_nq)))))
        nq = max(1, min(self.max_nq, nq))
        k = int(rng.choice(np.asarray(self.k_choices)))
        m = int(rng.integers(int(math.ceil(c.n / 10)), c.n + 1))
        if not hasattr(self, "_boxes"):
            self._boxes = [bbox_expanded(cc.points, 1.0) for cc in self.clouds]
        lo, hi = self._boxes[ci]
        return Request(ci, uniform_in_box(rng, nq, lo, hi), k, m)

    def deletion_plan(self, frac: float = 0.01, batch: int = 1000, parts: int = 1):
        """Per cloud, `frac` of its ranks without replacement, split into batches <= batch,
        in a seeded random order.  With parts > 1, returns that many such plans over
        disjoint rank sets (one per run that deletes from the same clouds)."""
        rng = np.random.default_rng(np.random.SeedSequence(7).spawn(1)[0])
        plans = [[] for _ in range(parts)]
        for ci, c in enumerate(self.clouds):
            cnt = int(round(frac * c.n))
            ranks = rng.choice(c.n, cnt * parts, replace=False).astype(np.int32)
            for p in range(parts):
                mine = ranks[p * cnt:(p + 1) * cnt]
                for s in range(0, cnt, batch):
                    plans[p].append((ci, mine[s:s + batch]))
        out = []
        for plan in plans:
            order = rng.permutation(len(plan))
            out.append([plan[i] for i in order])
        return out[0] if parts == 1 else out


def serving_clouds(num: int = 64, n_lo: int = 10_000, n_hi: int = 2_000_000,
                   noise: float = 1e-3, seed: int = 0) -> ServingWorkload:
    """`num` resident clouds, sizes log-uniform in [n_lo, n_hi], shapes as in many_clouds."""
    st = _streams(seed)
    sizes = np.rint(np.exp(st[S_SHAPE].uniform(math.log(n_lo), math.log(n_hi), num))).astype(int)
    shapes = st[S_SHAPE].integers(0, len(SHAPES), num)
    clouds = [_shape_cloud(st[S_POINTS], st[S_ORDER], st[S_SHAPE], int(sizes[i]),
                           SHAPES[shapes[i]], noise) for i in range(num)]
    return ServingWorkload(f"serving_{num}_clouds", clouds, st[S_REQ])


@dataclasses.dataclass
class DynamicWorkload:
    """The dynamic benchmark of Sec. 5.4 (after ikd-Tree's): start with n0
    points; every iteration inserts `insert_per_iter` points and answers `queries_per_iter`
    queries with k neighbours; every `delete_every` iterations `delete_count` random live
    points are deleted, every `batch_every` iterations `batch_count` more are inserted."""
    name: str
    points: np.ndarray          # float32 [N, 3], in insertion order (the stream)
    n0: int
    iterations: int
    insert_per_iter: int
    queries_per_iter: int
    k: int
    delete_every: int
    delete_count: int
    batch_every: int
    batch_count: int
    qlo: np.ndarray
    qhi: np.ndarray
    rng: np.random.Generator    # queries and deletion picks, drawn in iteration order


def dynamic_stream(scenario: str = "surface", iterations: int = 2000, seed: int = 0,
                   n0: int = 5000, insert_per_iter: int = 200, queries_per_iter: int = 2000,
                   k: int = 20, delete_every: int = 50, delete_count: int = 100,
                   batch_every: int = 100, batch_count: int = 2000) -> DynamicWorkload:
    """scenario "surface": points on the torus (normal noise 1e-3) standing in for a scanned
    model, queries uniform in the 2x bounding box; "volume": points and queries uniform in
    [-10, 10]^3."""
    st = _streams(seed)
    total = n0 + iterations * insert_per_iter + (iterations // batch_every) * batch_count
    if scenario == "surface":
        gen = lambda m: sample_torus(st[S_POINTS], m, 1e-3)
    elif scenario == "volume":
        gen = lambda m: st[S_POINTS].uniform(-10.0, 10.0, (m, 3))
    else:
        raise ValueError(scenario)
    p = _dedupe_f32(gen(total), gen)
    p = np.ascontiguousarray(p[st[S_ORDER].permutation(total)])
    if scenario == "surface":
        lo, hi = bbox_expanded(p, 2.0)
    else:
        lo, hi = np.full(3, -10.0), np.full(3, 10.0)
    return DynamicWorkload(f"dynamic_{scenario}", p, n0, iterations, insert_per_iter,
                           queries_per_iter, k, delete_every, delete_count, batch_every,
                           batch_count, lo, hi, st[S_REQ])


# --------------------------------------------------------------------------------------
# small helpers for tests
# --------------------------------------------------------------------------------------
def random_cloud(n: int, seed: int, shape: str = "sphere", noise: float = 1e-3) -> Cloud:
    st = _streams(seed)
    return _shape_cloud(st[S_POINTS], st[S_ORDER], st[S_SHAPE], n, shape, noise)


def lattice_cloud(side: int, seed: int, spacing: float = 1.0) -> Cloud:
    """side^3 integer-lattice points (massively cospherical/coplanar) in a random order."""
    g = np.arange(side, dtype=np.float32) * np.float32(spacing)
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    order = _streams(seed)[S_ORDER].permutation(p.shape[0]).astype(np.int32)
    return Cloud(np.ascontiguousarray(p), order, "lattice")
