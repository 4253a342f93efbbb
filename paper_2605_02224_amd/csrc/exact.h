// Exact geometric predicates for the host-side Delaunay construction.
//
// The successor lists are defined by Voronoi adjacency at insertion time (Sec. 3), so the
// triangulation that produces them must be exactly Delaunay.  Both predicates are evaluated
// first in double precision with a forward error bound; when the sign is not certified they
// are re-evaluated exactly with floating-point expansions: sums of non-overlapping doubles,
// built from the error-free transformations two_sum (Knuth) and two_prod (via FMA), as in
// the adaptive-precision arithmetic published by Priest and by Shewchuk.  This file is our
// own implementation of those textbook operations; compile with -ffp-contract=off.
//
// Conventions (all points are double triples):
//   orient3d(a,b,c,d) = det[b-a; c-a; d-a]            (> 0: d on the side of (b-a)x(c-a))
//   insphere(a,b,c,d,e) > 0 iff e lies strictly inside the circumsphere of a tetrahedron
//                             with orient3d(a,b,c,d) > 0.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace mknn {

// ---------------------------------------------------------------------------------------
// expansions: value = sum of components, components non-overlapping, increasing magnitude,
// zeros removed.  The sign of a non-empty expansion is the sign of its last component.
// ---------------------------------------------------------------------------------------
struct Expansion {
  std::vector<double> c;
  Expansion() {}
  explicit Expansion(double v) { if (v != 0.0) c.push_back(v); }
  int sign() const { return c.empty() ? 0 : (c.back() > 0 ? 1 : -1); }
  double approx() const { double s = 0; for (double v : c) s += v; return s; }
};

inline void two_sum(double a, double b, double &x, double &y) {
  x = a + b;
  double bv = x - a;
  double av = x - bv;
  double br = b - bv;
  double ar = a - av;
  y = ar + br;
}

inline void two_prod(double a, double b, double &x, double &y) {
  x = a * b;
  y = std::fma(a, b, -x);
}

// e + b; the running sum absorbs each component from the smallest up, emitting the
// rounding errors as the new low-order components.
inline Expansion grow(const Expansion &e, double b) {
  Expansion h;
  h.c.reserve(e.c.size() + 1);
  double q = b;
  for (double ei : e.c) {
    double s, err;
    two_sum(q, ei, s, err);
    if (err != 0.0) h.c.push_back(err);
    q = s;
  }
  if (q != 0.0) h.c.push_back(q);
  return h;
}

inline Expansion add(const Expansion &e, const Expansion &f) {
  Expansion h = e;
  for (double fi : f.c) h = grow(h, fi);
  return h;
}

inline Expansion negate(const Expansion &e) {
  Expansion h = e;
  for (double &v : h.c) v = -v;
  return h;
}

inline Expansion sub(const Expansion &e, const Expansion &f) { return add(e, negate(f)); }

inline Expansion scale(const Expansion &e, double b) {
  Expansion h;
  for (double ei : e.c) {
    double p, pe;
    two_prod(ei, b, p, pe);
    if (pe != 0.0) h = grow(h, pe);
    if (p != 0.0) h = grow(h, p);
  }
  return h;
}

inline Expansion mul(const Expansion &e, const Expansion &f) {
  Expansion h;
  for (double fj : f.c) h = add(h, scale(e, fj));
  return h;
}

// exact difference a - b of two doubles
inline Expansion diff(double a, double b) {
  double x, y;
  two_sum(a, -b, x, y);
  Expansion h;
  if (y != 0.0) h.c.push_back(y);
  if (x != 0.0) h.c.push_back(x);
  return h;
}

// ---------------------------------------------------------------------------------------
// exact determinants over expansions
// ---------------------------------------------------------------------------------------
inline Expansion det2(const Expansion &a, const Expansion &b, const Expansion &c,
                      const Expansion &d) {  // a*d - b*c
  return sub(mul(a, d), mul(b, c));
}

// det of rows u, v, w (each 3 expansions)
inline Expansion det3(const Expansion *u, const Expansion *v, const Expansion *w) {
  Expansion m0 = det2(v[1], v[2], w[1], w[2]);
  Expansion m1 = det2(v[0], v[2], w[0], w[2]);
  Expansion m2 = det2(v[0], v[1], w[0], w[1]);
  return add(sub(mul(u[0], m0), mul(u[1], m1)), mul(u[2], m2));
}

inline int orient3d_exact(const double *a, const double *b, const double *c, const double *d) {
  Expansion r[3][3];
  for (int k = 0; k < 3; ++k) {
    r[0][k] = diff(b[k], a[k]);
    r[1][k] = diff(c[k], a[k]);
    r[2][k] = diff(d[k], a[k]);
  }
  return det3(r[0], r[1], r[2]).sign();
}

// Forward error bound of the double evaluation below, in units of the permanent.  The
// textbook analysis gives 7 eps + O(eps^2) (eps = 2^-53); twice that is used as margin.
constexpr double kEps = 1.1102230246251565e-16;
constexpr double kOrientBound = 16.0 * kEps;
constexpr double kInsphereBound = 40.0 * kEps;

inline int orient3d(const double *a, const double *b, const double *c, const double *d) {
  double bx = b[0] - a[0], by = b[1] - a[1], bz = b[2] - a[2];
  double cx = c[0] - a[0], cy = c[1] - a[1], cz = c[2] - a[2];
  double dx = d[0] - a[0], dy = d[1] - a[1], dz = d[2] - a[2];
  double m0 = cy * dz - cz * dy;
  double m1 = cx * dz - cz * dx;
  double m2 = cx * dy - cy * dx;
  double det = bx * m0 - by * m1 + bz * m2;
  double perm = std::fabs(bx) * (std::fabs(cy * dz) + std::fabs(cz * dy)) +
                std::fabs(by) * (std::fabs(cx * dz) + std::fabs(cz * dx)) +
                std::fabs(bz) * (std::fabs(cx * dy) + std::fabs(cy * dx));
  double bound = kOrientBound * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return orient3d_exact(a, b, c, d);
}

// Lifted determinant: rows (X - e, |X - e|^2) for X = a, b, c, d; insphere = -det.
inline int insphere_exact(const double *a, const double *b, const double *c, const double *d,
                          const double *e) {
  const double *pts[4] = {a, b, c, d};
  Expansion r[4][3], lift[4];
  for (int i = 0; i < 4; ++i) {
    for (int k = 0; k < 3; ++k) r[i][k] = diff(pts[i][k], e[k]);
    lift[i] = add(add(mul(r[i][0], r[i][0]), mul(r[i][1], r[i][1])), mul(r[i][2], r[i][2]));
  }
  // cofactor expansion along the lift column: det = -L0 M0 + L1 M1 - L2 M2 + L3 M3
  Expansion M0 = det3(r[1], r[2], r[3]);
  Expansion M1 = det3(r[0], r[2], r[3]);
  Expansion M2 = det3(r[0], r[1], r[3]);
  Expansion M3 = det3(r[0], r[1], r[2]);
  Expansion det = add(sub(mul(lift[1], M1), mul(lift[0], M0)),
                      sub(mul(lift[3], M3), mul(lift[2], M2)));
  return -det.sign();
}

inline int insphere(const double *a, const double *b, const double *c, const double *d,
                    const double *e) {
  double r[4][3], L[4];
  const double *pts[4] = {a, b, c, d};
  for (int i = 0; i < 4; ++i) {
    for (int k = 0; k < 3; ++k) r[i][k] = pts[i][k] - e[k];
    L[i] = r[i][0] * r[i][0] + r[i][1] * r[i][1] + r[i][2] * r[i][2];
  }
  auto m3 = [&](int i, int j, int k, double &perm) {
    double m0 = r[j][1] * r[k][2] - r[j][2] * r[k][1];
    double m1 = r[j][0] * r[k][2] - r[j][2] * r[k][0];
    double m2 = r[j][0] * r[k][1] - r[j][1] * r[k][0];
    perm = std::fabs(r[i][0]) * (std::fabs(r[j][1] * r[k][2]) + std::fabs(r[j][2] * r[k][1])) +
           std::fabs(r[i][1]) * (std::fabs(r[j][0] * r[k][2]) + std::fabs(r[j][2] * r[k][0])) +
           std::fabs(r[i][2]) * (std::fabs(r[j][0] * r[k][1]) + std::fabs(r[j][1] * r[k][0]));
    return r[i][0] * m0 - r[i][1] * m1 + r[i][2] * m2;
  };
  double p0, p1, p2, p3;
  double M0 = m3(1, 2, 3, p0), M1 = m3(0, 2, 3, p1), M2 = m3(0, 1, 3, p2), M3 = m3(0, 1, 2, p3);
  double det = (L[1] * M1 - L[0] * M0) + (L[3] * M3 - L[2] * M2);
  double perm = L[0] * p0 + L[1] * p1 + L[2] * p2 + L[3] * p3;
  double bound = kInsphereBound * perm;
  if (det > bound) return -1;
  if (-det > bound) return 1;
  return insphere_exact(a, b, c, d, e);
}

// Sign of component k of (b-a) x (c-a), exactly.
inline int cross_component_sign(const double *a, const double *b, const double *c, int k) {
  int i = (k + 1) % 3, j = (k + 2) % 3;
  Expansion bi = diff(b[i], a[i]), bj = diff(b[j], a[j]);
  Expansion ci = diff(c[i], a[i]), cj = diff(c[j], a[j]);
  return det2(bi, bj, ci, cj).sign();
}

}  // namespace mknn
