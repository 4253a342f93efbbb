// Host half of the C ABI: construction of successor lists and host-side views.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "cloud.h"
#include "exact.h"

namespace mknn {

static thread_local std::string g_err;

mknn_status set_error(mknn_status s, const std::string &msg) {
  g_err = msg;
  return s;
}
void clear_error() { g_err.clear(); }

// Lists of clouds with fewer than four points (the Delaunay start needs four affinely
// independent sites).  Voronoi adjacency of 2 or 3 sites: all pairs, except that of three
// collinear sites the middle one separates the outer two.
static void tiny_lists(const std::vector<double> &P, int64_t n, Csr *succ) {
  std::vector<std::vector<int32_t>> L(n);
  if (n >= 2) L[0].push_back(1);
  if (n == 3) {
    const double *a = &P[0], *b = &P[3], *c = &P[6];
    bool collinear = true;
    for (int k = 0; k < 3; ++k) collinear &= cross_component_sign(a, b, c, k) == 0;
    auto between = [](const double *x, const double *lo, const double *hi) {
      // x strictly between lo and hi on their common line: (lo - x).(hi - x) < 0
      Expansion s;
      for (int k = 0; k < 3; ++k) s = add(s, mul(diff(lo[k], x[k]), diff(hi[k], x[k])));
      return s.sign() < 0;
    };
    bool adj02 = !(collinear && between(b, a, c));
    bool adj12 = !(collinear && between(a, b, c));
    if (adj02) L[0].push_back(2);
    if (adj12) L[1].push_back(2);
  }
  succ->off.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) succ->off[i + 1] = succ->off[i] + (int64_t)L[i].size();
  succ->ent.clear();
  for (int64_t i = 0; i < n; ++i) succ->ent.insert(succ->ent.end(), L[i].begin(), L[i].end());
}

static void transpose(const Csr &s, int64_t n, Csr *t) {
  t->off.assign(n + 1, 0);
  for (int32_t e : s.ent) t->off[e + 1]++;
  for (int64_t i = 0; i < n; ++i) t->off[i + 1] += t->off[i];
  t->ent.resize(s.ent.size());
  std::vector<int64_t> pos(t->off.begin(), t->off.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = s.off[i]; e < s.off[i + 1]; ++e) t->ent[pos[s.ent[e]]++] = (int32_t)i;
}

}  // namespace mknn

using namespace mknn;

extern "C" {

const char *mknn_last_error(void) { return g_err.c_str(); }

const char *mknn_version(void) { return "mknn-gfx950 0.1"; }

mknn_status mknn_build(const float *xyz, int64_t n, const int32_t *order, mknn_cloud **out) {
  clear_error();
  if (!out) return set_error(MKNN_EINVAL, "mknn_build: out is NULL");
  *out = nullptr;
  if (!xyz) return set_error(MKNN_EINVAL, "mknn_build: xyz is NULL");
  if (n < 1) return set_error(MKNN_EINVAL, "mknn_build: n must be >= 1");
  if (n > (int64_t)1 << 30) return set_error(MKNN_EUNSUPPORTED, "mknn_build: n above 2^30");
  mknn_cloud *c = nullptr;
  try {
    c = new mknn_cloud();
    c->n = n;
    c->order.resize(n);
    if (order) {
      std::vector<char> seen(n, 0);
      for (int64_t r = 0; r < n; ++r) {
        int32_t o = order[r];
        if (o < 0 || o >= n || seen[o]) {
          delete c;
          return set_error(MKNN_EINVAL, "mknn_build: order is not a permutation of 0..n-1");
        }
        seen[o] = 1;
        c->order[r] = o;
      }
    } else {
      for (int64_t r = 0; r < n; ++r) c->order[r] = (int32_t)r;
    }
    c->xyz.resize(3 * n);
    std::vector<double> P(3 * n);
    for (int64_t r = 0; r < n; ++r) {
      for (int k = 0; k < 3; ++k) {
        float v = xyz[3 * (int64_t)c->order[r] + k];
        if (!std::isfinite(v)) {
          delete c;
          return set_error(MKNN_ENONFINITE, "mknn_build: non-finite coordinate at point " +
                                                std::to_string(c->order[r]));
        }
        c->xyz[3 * r + k] = v;
        P[3 * r + k] = (double)v;
      }
    }
    for (int k = 0; k < 3; ++k) {
      c->lo[k] = c->hi[k] = c->xyz[k];
      for (int64_t r = 1; r < n; ++r) {
        c->lo[k] = std::min(c->lo[k], c->xyz[3 * r + k]);
        c->hi[k] = std::max(c->hi[k], c->xyz[3 * r + k]);
      }
    }
    if (n < 4) {
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
          if (P[3 * i] == P[3 * j] && P[3 * i + 1] == P[3 * j + 1] && P[3 * i + 2] == P[3 * j + 2]) {
            delete c;
            return set_error(MKNN_EDUPLICATE, "mknn_build: duplicate points");
          }
      tiny_lists(P, n, &c->succ);
    } else {
      DelaunayBuilder b(P.data(), n);
      int64_t bad = -1;
      BuildStatus s = b.build(&bad);
      if (s == kBuildDuplicate) {
        delete c;
        return set_error(MKNN_EDUPLICATE, "mknn_build: point " +
                                              std::to_string(c->order[bad]) +
                                              " duplicates an earlier point");
      }
      Csr succ;
      if (s == kBuildDegenerateStart) {
        // the first four ranks are coplanar: start from the first ranks off their line and
        // plane (or spare points off them) and record the lists of the low-dimensional prefix
        std::vector<double> P2(P);
        P2.resize(3 * (size_t)(n + 2));
        int32_t A = -1, B = -1;
        s = DelaunayBuilder::low_dim_plan(P2.data(), n, &A, &B, &bad);
        if (s == kBuildOk) {
          DelaunayBuilder b2(P2.data(), n + 2);
          s = b2.build_low_dim(n, A, B, &bad);
          if (s == kBuildOk) {
            succ = b2.successors();
            succ.off.resize(n + 1);   // the spare points own no entries
            succ.ent.resize(succ.off[n]);
          }
        }
        if (s == kBuildDuplicate) {
          delete c;
          return set_error(MKNN_EDUPLICATE, "mknn_build: point " +
                                                std::to_string(c->order[bad]) +
                                                " duplicates an earlier point");
        }
      } else if (s == kBuildOk) {
        succ = b.successors();
      }
      if (s != kBuildOk) {
        delete c;
        return set_error(MKNN_EUNSUPPORTED, "mknn_build: internal failure at rank " +
                                                std::to_string(bad));
      }
      c->succ = std::move(succ);
    }
    transpose(c->succ, n, &c->pred);
    c->live.assign(n, 1);
    c->nlive = n;
    c->head = 0;
  } catch (const std::bad_alloc &) {
    delete c;
    return set_error(MKNN_ENOMEM, "mknn_build: out of host memory");
  }
  *out = c;
  return MKNN_OK;
}

int64_t mknn_size(const mknn_cloud *c) { return c ? c->n.load() : 0; }

mknn_status mknn_successors(const mknn_cloud *c, const int64_t **offsets, const int32_t **ranks,
                            int64_t *nnz) {
  clear_error();
  if (!c || !offsets || !ranks || !nnz) return set_error(MKNN_EINVAL, "mknn_successors: NULL");
  refresh_csr(const_cast<mknn_cloud *>(c));
  *offsets = c->succ.off.data();
  *ranks = c->succ.ent.data();
  *nnz = (int64_t)c->succ.ent.size();
  return MKNN_OK;
}

mknn_status mknn_points_by_rank(const mknn_cloud *c, const float **xyz) {
  clear_error();
  if (!c || !xyz) return set_error(MKNN_EINVAL, "mknn_points_by_rank: NULL");
  *xyz = c->xyz.data();
  return MKNN_OK;
}

}  // extern "C"
