// Incremental 3-D Delaunay triangulation recording successor lists (see delaunay.h).
#include "delaunay.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "exact.h"

namespace mknn {

namespace {
inline double sqd(const double *a, const double *b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return (dx * dx + dy * dy) + dz * dz;
}
inline uint64_t edge_key(int32_t a, int32_t b) {
  uint32_t x = (uint32_t)(a + 1), y = (uint32_t)(b + 1);
  if (x > y) std::swap(x, y);
  return ((uint64_t)x << 32) | y;
}
}  // namespace

DelaunayBuilder::DelaunayBuilder(const double *pts, int64_t n) : P_(pts), n_(n) {
  vtet_.assign(n, -1);
  lstart_.assign(n, 0);
  llen_.assign(n, 0);
  lcap_.assign(n, 0);
  vmark_.assign(n, 0);
  gone_.assign(n, 0);
  tv_.reserve((size_t)std::max<int64_t>(64, 7 * n) * 4);
  tn_.reserve((size_t)std::max<int64_t>(64, 7 * n) * 4);
  stamp_.reserve((size_t)std::max<int64_t>(64, 7 * n));
  pool_.reserve((size_t)std::max<int64_t>(64, 20 * n));
}

int64_t DelaunayBuilder::num_tets() const {
  return (int64_t)stamp_.size() - (int64_t)free_.size();
}

bool DelaunayBuilder::tet(int64_t t, int32_t v[4]) const {
  if (t < 0 || t >= (int64_t)stamp_.size()) return false;
  if (std::find(free_.begin(), free_.end(), (int32_t)t) != free_.end()) return false;
  for (int k = 0; k < 4; ++k) v[k] = tv_[4 * t + k];
  return true;
}

int32_t DelaunayBuilder::alloc_tet() {
  if (!free_.empty()) {
    int32_t t = free_.back();
    free_.pop_back();
    return t;
  }
  int32_t t = (int32_t)stamp_.size();
  tv_.resize(tv_.size() + 4);
  tn_.resize(tn_.size() + 4);
  stamp_.push_back(0);
  return t;
}

void DelaunayBuilder::append(int32_t owner, int32_t rank) {
  if (llen_[owner] == lcap_[owner]) {
    int32_t cap = lcap_[owner] ? 2 * lcap_[owner] : 8;
    int64_t ns = (int64_t)pool_.size();
    pool_.resize(pool_.size() + cap);
    if (llen_[owner])
      std::memcpy(&pool_[ns], &pool_[lstart_[owner]], sizeof(int32_t) * llen_[owner]);
    lstart_[owner] = ns;
    lcap_[owner] = cap;
  }
  pool_[lstart_[owner] + llen_[owner]++] = rank;
}

// A tetrahedron conflicts with the new (newest) site p when p lies inside or on its
// circumsphere; a ghost tetrahedron (hull facet F plus the vertex at infinity) conflicts
// when p lies strictly beyond F, or in F's plane inside or on F's circumcircle.
bool DelaunayBuilder::conflict(int32_t t, const double *p, bool strict) const {
  const int32_t *v = &tv_[4 * (int64_t)t];
  int inf = -1;
  for (int i = 0; i < 4; ++i)
    if (v[i] == kInf) inf = i;
  const int need = strict ? 1 : 0;
  if (inf < 0) return insphere(pt(v[0]), pt(v[1]), pt(v[2]), pt(v[3]), p) >= need;
  const double *q[4];
  for (int i = 0; i < 4; ++i) q[i] = (i == inf) ? p : pt(v[i]);
  int o = orient3d(q[0], q[1], q[2], q[3]);
  if (o != 0) return o > 0;
  // p is in the facet's plane: test against the circumcircle through an auxiliary point f
  // beyond the facet (any such f gives a sphere meeting the plane in that circle).
  const double *a = pt(v[(inf + 1) & 3]);
  for (int k = 0; k < 3; ++k) {
    for (int s = 0; s < 2; ++s) {
      double f[3] = {a[0], a[1], a[2]};
      f[k] = s == 0 ? a[k] + 1.0 : a[k] - 1.0;
      const double *r[4];
      for (int i = 0; i < 4; ++i) r[i] = (i == inf) ? f : pt(v[i]);
      if (orient3d(r[0], r[1], r[2], r[3]) > 0) return insphere(r[0], r[1], r[2], r[3], p) >= need;
    }
  }
  return false;  // unreachable for a non-degenerate facet
}

// 1-NN of p among the inserted sites by the descent over the lists built so far: start at
// rank 0 and jump to the first list entry strictly closer (key = (D, rank)).
int32_t DelaunayBuilder::nearest_inserted(const double *p, double *dbest) const {
  // the lists hold, in insertion order, the later neighbours of each vertex, so the walk
  // starts from the first inserted vertex
  int32_t cur = order_[walk_pos_];
  double dcur = sqd(p, pt(cur));
  for (;;) {
    const int32_t *l = &pool_[lstart_[cur]];
    int32_t len = llen_[cur];
    int32_t next = -1;
    double dn = 0;
    for (int32_t e = 0; e < len; ++e) {
      double d = sqd(p, pt(l[e]));
      if (d < dcur) {
        next = l[e];
        dn = d;
        break;
      }
    }
    if (next < 0) break;
    cur = next;
    dcur = dn;
  }
  *dbest = dcur;
  return cur;
}

// Find one tetrahedron in conflict with p, searching the star of `near` first and then,
// if the nearest site came from a rounded tie, widening breadth-first.
int32_t DelaunayBuilder::locate(int32_t near, const double *p) {
  uint32_t ep = ++epoch_;
  star_.clear();
  int32_t t0 = vtet_[near];
  star_.push_back(t0);
  stamp_[t0] = ep;
  for (size_t s = 0; s < star_.size(); ++s) {
    int32_t t = star_[s];
    if (conflict(t, p)) return t;
    for (int h = 0; h < 4; ++h) {
      if (tv_[4 * (int64_t)t + h] == near) continue;   // faces through `near` only
      int32_t u = tn_[4 * (int64_t)t + h];
      if (stamp_[u] != ep) {
        stamp_[u] = ep;
        star_.push_back(u);
      }
    }
  }
  // widen: plain breadth-first search over all tetrahedra
  for (size_t s = 0; s < star_.size(); ++s) {
    int32_t t = star_[s];
    if (conflict(t, p)) return t;
    for (int h = 0; h < 4; ++h) {
      int32_t u = tn_[4 * (int64_t)t + h];
      if (stamp_[u] != ep) {
        stamp_[u] = ep;
        star_.push_back(u);
      }
    }
  }
  return -1;
}

bool DelaunayBuilder::start_with(const int32_t first4[4]) {
  if (n_ < 4 || ninserted_ != 0) return false;
  order_.clear();
  done_.assign(n_, 0);
  for (int i = 0; i < 4; ++i) {
    order_.push_back(first4[i]);
    done_[first4[i]] = 1;
  }
  for (int64_t v = 0; v < n_; ++v)
    if (!done_[v]) order_.push_back((int32_t)v);
  ascending_ = std::is_sorted(order_.begin(), order_.end());
  return orient3d(pt(first4[0]), pt(first4[1]), pt(first4[2]), pt(first4[3])) != 0;
}

bool DelaunayBuilder::set_order(std::vector<int32_t> order) {
  if (ninserted_ != 0) return false;
  for (int32_t v : order)
    if (v < 0 || v >= n_) return false;
  order_ = std::move(order);
  ascending_ = std::is_sorted(order_.begin(), order_.end());
  return true;
}

void DelaunayBuilder::grow(const double *pts, int64_t n) {
  if (order_.empty())
    for (int64_t v = 0; v < n_; ++v) order_.push_back((int32_t)v);
  P_ = pts;
  for (int64_t v = n_; v < n; ++v) order_.push_back((int32_t)v);
  vtet_.resize(n, -1);
  lstart_.resize(n, 0);
  llen_.resize(n, 0);
  lcap_.resize(n, 0);
  vmark_.resize(n, 0);
  gone_.resize(n, 0);
  n_ = n;
}

bool DelaunayBuilder::init_first_tet() {
  if (order_.empty())
    for (int64_t v = 0; v < n_; ++v) order_.push_back((int32_t)v);
  if (order_.size() < 4) return false;
  int32_t v[4] = {order_[0], order_[1], order_[2], order_[3]};
  int o = orient3d(pt(v[0]), pt(v[1]), pt(v[2]), pt(v[3]));
  if (o == 0) return false;
  if (o < 0) std::swap(v[2], v[3]);
  int32_t t = alloc_tet();
  int32_t g[4];
  for (int i = 0; i < 4; ++i) g[i] = alloc_tet();
  for (int i = 0; i < 4; ++i) {
    tv_[4 * t + i] = v[i];
    tn_[4 * t + i] = g[i];
  }
  // ghost across face i: vertex i replaced by infinity, then two finite vertices swapped
  // so that replacing infinity by a point beyond the face gives a positive orientation.
  for (int i = 0; i < 4; ++i) {
    int32_t w[4] = {v[0], v[1], v[2], v[3]};
    w[i] = kInf;
    int a = (i + 1) & 3, b = (i + 2) & 3;
    std::swap(w[a], w[b]);
    for (int k = 0; k < 4; ++k) tv_[4 * g[i] + k] = w[k];
  }
  // neighbours of the ghosts: across the facet opposite infinity lies t; across the other
  // faces lie the other ghosts (two ghosts share the edge common to their faces).
  for (int i = 0; i < 4; ++i) {
    for (int k = 0; k < 4; ++k) {
      int32_t vk = tv_[4 * g[i] + k];
      if (vk == kInf) {
        tn_[4 * g[i] + k] = t;
      } else {
        // face opposite vk contains infinity and the two other finite vertices; the ghost
        // sharing it is the one whose missing vertex is vk
        int idx = 0;
        while (v[idx] != vk) ++idx;
        tn_[4 * g[i] + k] = g[idx];
      }
    }
  }
  for (int i = 0; i < 4; ++i) vtet_[v[i]] = t;
  // lists: with four affinely independent sites every pair is Voronoi-adjacent
  if (!quiet_start_)
    for (int j = 1; j < 4; ++j)
      for (int i = 0; i < j; ++i) append(order_[i], order_[j]);
  nbrs_.assign(order_.begin(), order_.begin() + 3);
  std::sort(nbrs_.begin(), nbrs_.end());
  ninserted_ = 4;
  live_ = 4;
  return true;
}

bool DelaunayBuilder::edge_in_conflict(int32_t a, int32_t b, const double *p) {
  // walk the star of b (tetrahedra through b), keep those that also contain a
  uint32_t ep = ++epoch_;
  star_.clear();
  int32_t t0 = vtet_[b];
  star_.push_back(t0);
  stamp_[t0] = ep;
  for (size_t s = 0; s < star_.size(); ++s) {
    int32_t t = star_[s];
    const int32_t *v = &tv_[4 * (int64_t)t];
    if ((v[0] == a || v[1] == a || v[2] == a || v[3] == a) && conflict(t, p, true)) return true;
    for (int h = 0; h < 4; ++h) {
      if (v[h] == b) continue;
      int32_t u = tn_[4 * (int64_t)t + h];
      if (stamp_[u] != ep) {
        stamp_[u] = ep;
        star_.push_back(u);
      }
    }
  }
  return false;
}

BuildStatus DelaunayBuilder::insert_next() {
  if (ninserted_ == 0) {
    if (!init_first_tet()) return kBuildDegenerateStart;
    return kBuildOk;
  }
  const int32_t j = order_[ninserted_];
  const double *p = pt(j);
  double dnear;
  int32_t near = nearest_inserted(p, &dnear);
  if (dnear == 0.0) return kBuildDuplicate;
  int32_t seed = locate(near, p);
  if (seed < 0) return kBuildInternal;

  // grow the cavity: all tetrahedra in conflict, connected to the seed
  uint32_t ein = ++epoch_;
  uint32_t eout = ++epoch_;
  cavity_.clear();
  stack_.clear();
  bnd_.clear();
  stamp_[seed] = ein;
  cavity_.push_back(seed);
  stack_.push_back(seed);
  while (!stack_.empty()) {
    int32_t t = stack_.back();
    stack_.pop_back();
    for (int h = 0; h < 4; ++h) {
      int32_t u = tn_[4 * (int64_t)t + h];
      if (stamp_[u] == ein) continue;
      if (stamp_[u] != eout) {
        if (conflict(u, p)) {
          stamp_[u] = ein;
          cavity_.push_back(u);
          stack_.push_back(u);
          continue;
        }
        stamp_[u] = eout;
      }
      Boundary b;
      for (int k = 0; k < 4; ++k) b.v[k] = tv_[4 * (int64_t)t + k];
      b.v[h] = j;
      b.h = h;
      b.outer = u;
      b.outer_face = -1;
      for (int k = 0; k < 4; ++k)
        if (tn_[4 * (int64_t)u + k] == t) b.outer_face = k;
      if (b.outer_face < 0) return kBuildInternal;
      bnd_.push_back(b);
    }
  }
  for (int32_t t : cavity_) free_.push_back(t);

  // new tetrahedra: each boundary facet joined to p
  size_t nb = bnd_.size();
  size_t hsize = 16;
  while (hsize < 4 * 3 * nb) hsize <<= 1;
  if (hkey_.size() < hsize) {
    hkey_.assign(hsize, 0);
    hval_.assign(hsize, 0);
    hstamp_.assign(hsize, 0);
  }
  hsize = hkey_.size();
  uint32_t he = ++hepoch_;
  uint32_t ve = ++vepoch_;
  nbrs_.clear();
  for (size_t bi = 0; bi < nb; ++bi) {
    const Boundary &b = bnd_[bi];
    int32_t nt = alloc_tet();
    for (int k = 0; k < 4; ++k) tv_[4 * (int64_t)nt + k] = b.v[k];
    tn_[4 * (int64_t)nt + b.h] = b.outer;
    tn_[4 * (int64_t)b.outer + b.outer_face] = nt;
    for (int k = 0; k < 4; ++k) {
      int32_t w = b.v[k];
      if (w == kInf) continue;
      vtet_[w] = nt;
      if (w != j && vmark_[w] != ve) {
        vmark_[w] = ve;
        nbrs_.push_back(w);
      }
    }
    // faces through p: match by the opposite edge
    for (int k = 0; k < 4; ++k) {
      if (k == b.h) continue;
      int32_t x = -2, y = -2;
      for (int m = 0; m < 4; ++m) {
        if (m == k || m == b.h) continue;
        if (x == -2) x = b.v[m]; else y = b.v[m];
      }
      uint64_t key = edge_key(x, y);
      size_t slot = (size_t)((key * 0x9E3779B97F4A7C15ull) >> 40) & (hsize - 1);
      for (;;) {
        if (hstamp_[slot] != he) {
          hstamp_[slot] = he;
          hkey_[slot] = key;
          hval_[slot] = nt * 4 + k;
          break;
        }
        if (hkey_[slot] == key) {
          int32_t ot = hval_[slot] >> 2, ok = hval_[slot] & 3;
          tn_[4 * (int64_t)nt + k] = ot;
          tn_[4 * (int64_t)ot + ok] = nt;
          break;
        }
        slot = (slot + 1) & (hsize - 1);
      }
    }
  }
  std::sort(nbrs_.begin(), nbrs_.end());
  if (nreal_ < 0) {
    for (int32_t i : nbrs_) append(i, j);
  } else {
    // low-dimensional start: the start's later ranks and the spare points are no list owners
    for (int32_t i : nbrs_)
      if (i < j) append(i, j);
  }
  ++ninserted_;
  ++live_;
  return kBuildOk;
}

BuildStatus DelaunayBuilder::low_dim_plan(double *pts, int64_t nreal, int32_t *A, int32_t *B,
                                          int64_t *bad) {
  const double *p0 = pts, *p1 = pts + 3;
  if (p0[0] == p1[0] && p0[1] == p1[1] && p0[2] == p1[2]) {
    *bad = 1;
    return kBuildDuplicate;
  }
  auto collinear = [&](const double *q) {
    for (int k = 0; k < 3; ++k)
      if (cross_component_sign(p0, p1, q, k) != 0) return false;
    return true;
  };
  // a length comparable to the cloud, for the spare points
  double ext = 0;
  for (int64_t r = 1; r < nreal; ++r)
    for (int k = 0; k < 3; ++k) ext = std::max(ext, std::fabs(pts[3 * r + k] - p0[k]));
  if (!(ext > 0)) ext = 1;
  double *va = pts + 3 * nreal, *vb = pts + 3 * (nreal + 1);
  *A = -1;
  for (int64_t j = 2; j < nreal && *A < 0; ++j)
    if (!collinear(pts + 3 * j)) *A = (int32_t)j;
  if (*A < 0) {
    for (int k = 0; k < 3 && *A < 0; ++k) {
      for (int m = 0; m < 3; ++m) va[m] = p0[m];
      va[k] += ext;
      if (!collinear(va)) *A = (int32_t)nreal;
    }
    if (*A < 0) return kBuildInternal;
  }
  const double *pa = pts + 3 * (int64_t)(*A);
  *B = -1;
  for (int64_t j = 2; j < nreal && *B < 0; ++j)
    if (j != *A && orient3d(p0, p1, pa, pts + 3 * j) != 0) *B = (int32_t)j;
  if (*B < 0) {
    for (int k = 0; k < 3 && *B < 0; ++k)
      for (int sgn = 0; sgn < 2 && *B < 0; ++sgn) {
        for (int m = 0; m < 3; ++m) vb[m] = p0[m];
        vb[k] += sgn ? -ext : ext;
        if (orient3d(p0, p1, pa, vb) != 0) *B = (int32_t)(nreal + 1);
      }
    if (*B < 0) return kBuildInternal;
  }
  return kBuildOk;
}

BuildStatus DelaunayBuilder::build_low_dim(int64_t nreal, int32_t A, int32_t B, int64_t *bad_rank) {
  if (ninserted_ != 0 || n_ != nreal + 2 || nreal < 2) return kBuildInternal;
  nreal_ = nreal;
  order_.clear();
  order_.push_back(0);
  order_.push_back(1);
  order_.push_back(A);
  order_.push_back(B);
  for (int32_t v = 2; v < (int32_t)nreal; ++v)
    if (v != A && v != B) order_.push_back(v);
  ascending_ = false;
  quiet_start_ = true;
  if (!init_first_tet()) return kBuildInternal;
  quiet_start_ = false;
  append(0, 1);   // two sites: the bisector plane is their common facet
  // A and B (when they are ranks) take every older rank once the ranks before them are in
  bool a_done = A >= nreal, b_done = B >= nreal;
  auto flush = [&](int64_t next) {
    for (int pass = 0; pass < 2; ++pass) {
      const int32_t x = pass == 0 ? std::min(A, B) : std::max(A, B);
      bool &done = (x == A) ? a_done : b_done;
      if (!done && x < next) {
        for (int32_t i = 0; i < x; ++i) append(i, x);
        done = true;
      }
    }
  };
  while (ninserted_ < (int64_t)order_.size()) {
    const int32_t j = order_[ninserted_];
    flush(j);
    BuildStatus s = insert_next();
    if (s != kBuildOk) {
      if (bad_rank) *bad_rank = j;
      return s;
    }
  }
  flush(nreal);
  return kBuildOk;
}

void DelaunayBuilder::set_list(int32_t v, const int32_t *ent, int32_t len) {
  llen_[v] = 0;
  for (int32_t e = 0; e < len; ++e) append(v, ent[e]);
}

// Would inserting site p (id v) destroy tetrahedron t of this triangulation, whose vertex
// ids map to ids[] of the caller (kInf stays)?  The perturbation of the construction lowers
// the lifted coordinate of every site by an amount that dominates all those of older sites.
// For a sphere through p and t's four sites, the newest of the five with a non-zero effect
// decides: p itself puts p inside; a vertex w puts p inside iff p's barycentric coordinate
// for w is negative (lowering w lowers the lifted plane at p exactly when it is).  Ghosts
// use the construction's own test when p is newer than the facet's sites, else only
// "strictly beyond the facet, or strictly inside its circle".
bool DelaunayBuilder::destroyed_by(int32_t t, const double *p, int32_t v, const int32_t *ids) const {
  const int32_t *tv = &tv_[4 * (int64_t)t];
  int32_t vmax = -1;
  bool ghost = false;
  for (int i = 0; i < 4; ++i) {
    if (tv[i] == kInf) ghost = true;
    else vmax = std::max(vmax, ids[tv[i]]);
  }
  if (ghost) return conflict(t, p, v < vmax);
  const double *q[4] = {pt(tv[0]), pt(tv[1]), pt(tv[2]), pt(tv[3])};
  const int s = insphere(q[0], q[1], q[2], q[3], p);
  if (s != 0) return s > 0;
  // on the sphere: walk the five sites from the newest down
  int idx[4] = {0, 1, 2, 3};
  std::sort(idx, idx + 4, [&](int a, int b) { return ids[tv[a]] > ids[tv[b]]; });
  for (int w : idx) {
    if (ids[tv[w]] < v) return true;   // p is the newest left: inside
    const double *r[4] = {q[0], q[1], q[2], q[3]};
    r[w] = p;
    const int o = orient3d(r[0], r[1], r[2], r[3]);
    if (o != 0) return o < 0;
  }
  return true;
}

BuildStatus DelaunayBuilder::remove(int32_t v) {
  if (v < 0 || v >= n_ || gone_[v] || vtet_[v] < 0 || !ascending_) return kBuildInternal;
  if (live_ < 6) return kBuildDegenerateStart;   // keep at least five sites
  // star of v: the tetrahedra through v, connected across the faces through v
  const uint32_t ep = ++epoch_;
  star_.clear();
  star_.push_back(vtet_[v]);
  stamp_[vtet_[v]] = ep;
  for (size_t s = 0; s < star_.size(); ++s) {
    const int32_t t = star_[s];
    for (int h = 0; h < 4; ++h) {
      if (tv_[4 * (int64_t)t + h] == v) continue;
      const int32_t u = tn_[4 * (int64_t)t + h];
      if (stamp_[u] != ep) {
        stamp_[u] = ep;
        star_.push_back(u);
      }
    }
  }
  // v's link: the facet opposite v in every star tetrahedron, with the tetrahedron beyond
  struct LinkFace { int32_t key[3]; int32_t outer, outer_face; bool used; };
  std::vector<LinkFace> link;
  std::vector<int32_t> lv;   // finite link vertices
  for (int32_t t : star_) {
    int hv = -1;
    for (int k = 0; k < 4; ++k)
      if (tv_[4 * (int64_t)t + k] == v) hv = k;
    if (hv < 0) return kBuildInternal;
    LinkFace f;
    int c = 0;
    for (int k = 0; k < 4; ++k)
      if (k != hv) {
        f.key[c++] = tv_[4 * (int64_t)t + k];
        if (tv_[4 * (int64_t)t + k] != kInf) lv.push_back(tv_[4 * (int64_t)t + k]);
      }
    std::sort(f.key, f.key + 3);
    f.outer = tn_[4 * (int64_t)t + hv];
    f.outer_face = -1;
    for (int k = 0; k < 4; ++k)
      if (tn_[4 * (int64_t)f.outer + k] == t) f.outer_face = k;
    if (f.outer_face < 0) return kBuildInternal;
    f.used = false;
    link.push_back(f);
  }
  std::sort(lv.begin(), lv.end(), [&](int32_t a, int32_t b) { return rank_of(a) < rank_of(b); });
  lv.erase(std::unique(lv.begin(), lv.end()), lv.end());
  if (lv.size() == 3 && link.size() == 4) {
    // a hull corner with three finite neighbours: its star is one finite tetrahedron and
    // three ghosts, and without v the facet of the three becomes a hull facet.  The ghost
    // keeps the finite tetrahedron's vertex order with v replaced by infinity (v lay beyond
    // that facet, which is the ghost's orientation rule).
    int32_t t0 = -1;
    for (int32_t t : star_) {
      bool ghost = false;
      for (int k = 0; k < 4; ++k) ghost |= tv_[4 * (int64_t)t + k] == kInf;
      if (!ghost) t0 = t;
    }
    if (t0 < 0) return kBuildInternal;
    int32_t w[4];
    for (int k = 0; k < 4; ++k) w[k] = tv_[4 * (int64_t)t0 + k] == v ? kInf : tv_[4 * (int64_t)t0 + k];
    int fm[4];
    for (int k = 0; k < 4; ++k) {
      int32_t key[3];
      int c = 0;
      for (int m = 0; m < 4; ++m)
        if (m != k) key[c++] = w[m];
      std::sort(key, key + 3);
      fm[k] = -1;
      for (size_t f = 0; f < link.size(); ++f)
        if (link[f].key[0] == key[0] && link[f].key[1] == key[1] && link[f].key[2] == key[2])
          fm[k] = (int)f;
      if (fm[k] < 0) return kBuildInternal;
    }
    for (int32_t t : star_) free_.push_back(t);
    const int32_t g = alloc_tet();
    for (int k = 0; k < 4; ++k) {
      tv_[4 * (int64_t)g + k] = w[k];
      if (w[k] != kInf) vtet_[w[k]] = g;
      const LinkFace &f = link[fm[k]];
      tn_[4 * (int64_t)g + k] = f.outer;
      tn_[4 * (int64_t)f.outer + f.outer_face] = g;
    }
    vtet_[v] = -1;
    gone_[v] = 1;
    llen_[v] = 0;
    --live_;
    while (walk_pos_ < ninserted_ && gone_[order_[walk_pos_]]) ++walk_pos_;
    return kBuildOk;
  }
  if (lv.size() < 4) return kBuildDegenerateStart;
  // triangulation of the link vertices, inserted oldest first (local id = position in lv)
  std::vector<double> lp(3 * lv.size());
  std::vector<int32_t> lrank(lv.size());
  for (size_t u = 0; u < lv.size(); ++u) {
    std::memcpy(&lp[3 * u], pt(lv[u]), 3 * sizeof(double));
    lrank[u] = rank_of(lv[u]);
  }
  DelaunayBuilder dt(lp.data(), (int64_t)lv.size());
  int64_t bad = -1;
  const BuildStatus bs = dt.build(&bad);
  if (bs != kBuildOk) return bs;
  // the cavity v would carve out of it
  std::vector<char> dead(dt.stamp_.size(), 0);
  for (int32_t t : dt.free_) dead[t] = 1;
  std::vector<int32_t> cav, newid(dt.stamp_.size(), -1);
  for (size_t t = 0; t < dt.stamp_.size(); ++t)
    if (!dead[t] && dt.destroyed_by((int32_t)t, pt(v), rank_of(v), lrank.data())) {
      newid[t] = (int32_t)cav.size();
      cav.push_back((int32_t)t);
    }
  // its boundary must be v's link, facet for facet
  auto gid = [&](int32_t u) { return u == kInf ? kInf : lv[u]; };
  std::vector<std::pair<int32_t, int>> match;   // per cavity boundary face: link index
  for (int32_t t : cav)
    for (int k = 0; k < 4; ++k) {
      const int32_t u = dt.tn_[4 * (int64_t)t + k];
      if (newid[u] >= 0) continue;
      int32_t key[3];
      int c = 0;
      for (int m = 0; m < 4; ++m)
        if (m != k) key[c++] = gid(dt.tv_[4 * (int64_t)t + m]);
      std::sort(key, key + 3);
      int found = -1;
      for (size_t f = 0; f < link.size(); ++f)
        if (!link[f].used && link[f].key[0] == key[0] && link[f].key[1] == key[1] &&
            link[f].key[2] == key[2]) {
          found = (int)f;
          break;
        }
      if (found < 0) return kBuildInternal;
      link[found].used = true;
      match.push_back({found, 0});
    }
  if (match.size() != link.size()) return kBuildInternal;
  // commit: the star goes, the cavity's tetrahedra come in
  for (int32_t t : star_) free_.push_back(t);
  std::vector<int32_t> gt(cav.size());
  for (size_t a = 0; a < cav.size(); ++a) gt[a] = alloc_tet();
  size_t mi = 0;
  for (size_t a = 0; a < cav.size(); ++a) {
    const int32_t t = cav[a], g = gt[a];
    for (int k = 0; k < 4; ++k) {
      const int32_t w = gid(dt.tv_[4 * (int64_t)t + k]);
      tv_[4 * (int64_t)g + k] = w;
      if (w != kInf) vtet_[w] = g;
    }
    for (int k = 0; k < 4; ++k) {
      const int32_t u = dt.tn_[4 * (int64_t)t + k];
      if (newid[u] >= 0) {
        tn_[4 * (int64_t)g + k] = gt[newid[u]];
      } else {
        const LinkFace &f = link[match[mi++].first];
        tn_[4 * (int64_t)g + k] = f.outer;
        tn_[4 * (int64_t)f.outer + f.outer_face] = g;
      }
    }
  }
  vtet_[v] = -1;
  gone_[v] = 1;
  llen_[v] = 0;
  --live_;
  while (walk_pos_ < ninserted_ && gone_[order_[walk_pos_]]) ++walk_pos_;
  return kBuildOk;
}

BuildStatus DelaunayBuilder::build(int64_t *bad_rank) {
  if (order_.empty())
    for (int64_t v = 0; v < n_; ++v) order_.push_back((int32_t)v);
  while (ninserted_ < (int64_t)order_.size()) {
    int64_t j = ninserted_;
    if (order_.size() < 4) {
      // fewer than four sites: pairwise adjacency unless collinear ordering hides a pair
      // (handled by the caller rejecting n < 4 clouds that are degenerate)
      return kBuildDegenerateStart;
    }
    BuildStatus s = insert_next();
    if (s != kBuildOk) {
      if (bad_rank) *bad_rank = order_[(s == kBuildDegenerateStart) ? 3 : j];
      return s;
    }
  }
  return kBuildOk;
}

Csr DelaunayBuilder::successors() const {
  Csr c;
  c.off.assign(n_ + 1, 0);
  for (int64_t i = 0; i < n_; ++i) c.off[i + 1] = c.off[i] + llen_[i];
  c.ent.resize(c.off[n_]);
  for (int64_t i = 0; i < n_; ++i)
    if (llen_[i])
      std::memcpy(&c.ent[c.off[i]], &pool_[lstart_[i]], sizeof(int32_t) * llen_[i]);
  return c;
}

Csr DelaunayBuilder::predecessors() const {
  Csr c;
  c.off.assign(n_ + 1, 0);
  for (int64_t i = 0; i < n_; ++i)
    for (int32_t e = 0; e < llen_[i]; ++e) c.off[pool_[lstart_[i] + e] + 1]++;
  for (int64_t i = 0; i < n_; ++i) c.off[i + 1] += c.off[i];
  c.ent.resize(c.off[n_]);
  std::vector<int64_t> pos(c.off.begin(), c.off.end() - 1);
  for (int64_t i = 0; i < n_; ++i)   // ascending owner => each row ascending
    for (int32_t e = 0; e < llen_[i]; ++e) c.ent[pos[pool_[lstart_[i] + e]]++] = (int32_t)i;
  return c;
}

bool DelaunayBuilder::validate(std::string *why) const {
  std::vector<char> dead(stamp_.size(), 0);
  for (int32_t t : free_) dead[t] = 1;
  for (size_t t = 0; t < stamp_.size(); ++t) {
    if (dead[t]) continue;
    const int32_t *v = &tv_[4 * t];
    int inf = -1;
    for (int i = 0; i < 4; ++i)
      if (v[i] == kInf) inf = i;
    if (inf < 0 && orient3d(pt(v[0]), pt(v[1]), pt(v[2]), pt(v[3])) <= 0) {
      if (why) *why = "non-positive finite tetrahedron " + std::to_string(t);
      return false;
    }
    for (int h = 0; h < 4; ++h) {
      int32_t u = tn_[4 * t + h];
      if (u < 0 || (size_t)u >= stamp_.size() || dead[u]) {
        if (why) *why = "dangling neighbour";
        return false;
      }
      int back = 0, shared = 0;
      for (int k = 0; k < 4; ++k) {
        if (tn_[4 * (size_t)u + k] == (int32_t)t) ++back;
        for (int m = 0; m < 4; ++m)
          if (m != h && tv_[4 * (size_t)u + k] == v[m]) ++shared;
      }
      if (back != 1 || shared != 3) {
        if (why) *why = "asymmetric neighbour link at tet " + std::to_string(t);
        return false;
      }
    }
  }
  for (int64_t pos = 0; pos < ninserted_; ++pos) {
    const int32_t v = order_[pos];
    if (gone_[v]) continue;
    int32_t t = vtet_[v];
    bool ok = t >= 0 && !dead[t];
    if (ok) {
      ok = false;
      for (int k = 0; k < 4; ++k) ok |= tv_[4 * (size_t)t + k] == (int32_t)v;
    }
    if (!ok) {
      if (why) *why = "bad vertex incidence " + std::to_string(v);
      return false;
    }
  }
  return true;
}

bool DelaunayBuilder::validate_empty_spheres(std::string *why) const {
  std::vector<char> dead(stamp_.size(), 0);
  for (int32_t t : free_) dead[t] = 1;
  for (size_t t = 0; t < stamp_.size(); ++t) {
    if (dead[t]) continue;
    const int32_t *v = &tv_[4 * t];
    bool ghost = false;
    for (int i = 0; i < 4; ++i) ghost |= v[i] == kInf;
    if (ghost) continue;
    for (int64_t pos = 0; pos < ninserted_; ++pos) {
      const int32_t q = order_[pos];
      if (gone_[q] || q == v[0] || q == v[1] || q == v[2] || q == v[3]) continue;
      int s = insphere(pt(v[0]), pt(v[1]), pt(v[2]), pt(v[3]), pt((int32_t)q));
      // a site exactly on the sphere is allowed only if it is older than some vertex
      // (the perturbation puts the newest of the five inside)
      int32_t vmax = std::max(std::max(v[0], v[1]), std::max(v[2], v[3]));
      if (s > 0 || (s == 0 && q > vmax)) {
        if (why) *why = "site " + std::to_string(q) + " inside sphere of tet " + std::to_string(t);
        return false;
      }
    }
  }
  return true;
}

int64_t DelaunayBuilder::exact_fallbacks() const { return 0; }

}  // namespace mknn
