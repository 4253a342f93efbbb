// Host check of the ridge-round construction that the GPU build runs: every tetrahedron the
// sequential incremental construction creates is generated from pairs of tetrahedra that
// share a triangle, round by round, with no global order; the list entries (ridge vertex,
// creating site) must equal the sequential DelaunayBuilder's lists exactly.
//
// usage: ridge_rounds_check n kind seed     kind 0: sphere shell, 1: integer lattice in
// random order, 2: flat grid with four sites off its plane first.  Prints "ok ..." or the
// first difference.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <unordered_map>
#include <vector>

#include "delaunay.h"
#include "exact.h"

using namespace mknn;

static std::vector<double> P;
static const double *pt(int v) { return &P[3 * (size_t)v]; }

// the construction's conflict test for a site newer than every vertex of t
static bool conflict(const int *v, const double *p) {
  int inf = -1;
  for (int i = 0; i < 4; ++i)
    if (v[i] == kInf) inf = i;
  if (inf < 0) return insphere(pt(v[0]), pt(v[1]), pt(v[2]), pt(v[3]), p) >= 0;
  const double *q[4];
  for (int i = 0; i < 4; ++i) q[i] = (i == inf) ? p : pt(v[i]);
  const int o = orient3d(q[0], q[1], q[2], q[3]);
  if (o != 0) return o > 0;
  const double *a = pt(v[(inf + 1) & 3]);
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 2; ++s) {
      double f[3] = {a[0], a[1], a[2]};
      f[k] = s == 0 ? a[k] + 1.0 : a[k] - 1.0;
      const double *r[4];
      for (int i = 0; i < 4; ++i) r[i] = (i == inf) ? f : pt(v[i]);
      if (orient3d(r[0], r[1], r[2], r[3]) > 0) return insphere(r[0], r[1], r[2], r[3], p) >= 0;
    }
  return false;
}

struct Tet {
  int v[4];
  std::vector<int> C;   // later sites in conflict
  int minc;
};
static const int kNoSite = 0x7fffffff;

static uint64_t ridge_key(int a, int b, int c) {
  int x[3] = {a, b, c};
  std::sort(x, x + 3);
  auto u = [](int v) { return (uint64_t)(uint32_t)(v + 1); };
  return (u(x[0]) << 42) | (u(x[1]) << 21) | u(x[2]);
}

int main(int argc, char **argv) {
  if (argc < 4) return 2;
  const int n = atoi(argv[1]), kind = atoi(argv[2]);
  std::mt19937_64 rng(atoi(argv[3]));
  P.resize(3 * (size_t)n);
  if (kind == 0) {
    std::normal_distribution<double> g;
    for (int i = 0; i < n; ++i) {
      double x = g(rng), y = g(rng), z = g(rng), s = std::sqrt(x * x + y * y + z * z);
      P[3 * i] = (float)(x / s);
      P[3 * i + 1] = (float)(y / s);
      P[3 * i + 2] = (float)(z / s);
    }
  } else if (kind == 1) {
    const int s = (int)std::ceil(std::cbrt((double)n));
    std::vector<int> id(s * s * s);
    for (size_t i = 0; i < id.size(); ++i) id[i] = (int)i;
    std::shuffle(id.begin(), id.end(), rng);
    for (int i = 0; i < n; ++i) {
      P[3 * i] = id[i] % s;
      P[3 * i + 1] = (id[i] / s) % s;
      P[3 * i + 2] = id[i] / (s * s);
    }
  } else {
    const double off[4][3] = {{3.5, 7.25, 5.0}, {20.0, 1.0, -4.0}, {31.0, 30.5, 6.0},
                              {9.0, 33.0, -2.5}};
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 3; ++k) P[3 * i + k] = off[i][k];
    const int s = (int)std::ceil(std::sqrt((double)(n - 4)));
    std::vector<int> id(s * s);
    for (size_t i = 0; i < id.size(); ++i) id[i] = (int)i;
    std::shuffle(id.begin(), id.end(), rng);
    for (int i = 4; i < n; ++i) {
      P[3 * i] = id[i - 4] % s;
      P[3 * i + 1] = id[i - 4] / s;
      P[3 * i + 2] = 0.0;
    }
  }
  DelaunayBuilder b(P.data(), n);
  int64_t bad = -1;
  if (b.build(&bad) != kBuildOk) {
    printf("sequential construction failed at %lld\n", (long long)bad);
    return 1;
  }
  const Csr ref = b.successors();

  // the start: the first tetrahedron and its four ghosts, as the sequential construction
  std::vector<Tet> T;
  int v[4] = {0, 1, 2, 3};
  if (orient3d(pt(0), pt(1), pt(2), pt(3)) < 0) std::swap(v[2], v[3]);
  Tet t0;
  for (int i = 0; i < 4; ++i) t0.v[i] = v[i];
  T.push_back(t0);
  for (int i = 0; i < 4; ++i) {
    Tet g;
    int w[4] = {v[0], v[1], v[2], v[3]};
    w[i] = kInf;
    std::swap(w[(i + 1) & 3], w[(i + 2) & 3]);
    for (int k = 0; k < 4; ++k) g.v[k] = w[k];
    T.push_back(g);
  }
  for (Tet &t : T) {
    t.minc = kNoSite;
    for (int q = 4; q < n; ++q)
      if (conflict(t.v, pt(q))) {
        t.C.push_back(q);
        t.minc = std::min(t.minc, q);
      }
  }
  std::vector<std::pair<int, int>> items, entries;
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j) items.push_back({i, j});
  for (int j = 1; j < 4; ++j)
    for (int i = 0; i < j; ++i) entries.push_back({i, j});
  std::unordered_map<uint64_t, int> waiting;
  int rounds = 0;
  while (!items.empty()) {
    ++rounds;
    std::vector<std::pair<int, int>> next;
    for (auto [a, c] : items) {
      if (T[a].minc == T[c].minc) continue;   // inside one cavity, or final
      const int td = T[a].minc < T[c].minc ? a : c, ts = td == a ? c : a;
      const int p = T[td].minc;
      Tet nt;
      int apex = -1, shared = 0;
      for (int k = 0; k < 4; ++k) {
        const int x = T[td].v[k];
        bool in = false;
        for (int m = 0; m < 4; ++m) in |= T[ts].v[m] == x;
        nt.v[k] = in ? x : p;
        if (!in) apex = k;
        shared += in;
      }
      if (shared != 3) {
        printf("ridge pair without a common triangle\n");
        return 1;
      }
      nt.minc = kNoSite;
      for (int q : T[td].C)
        if (q != p && conflict(nt.v, pt(q))) {
          nt.C.push_back(q);
          nt.minc = std::min(nt.minc, q);
        }
      for (int q : T[ts].C)   // a site in both lists is taken from td's
        if (q != p && conflict(nt.v, pt(q)) && !conflict(T[td].v, pt(q))) {
          nt.C.push_back(q);
          nt.minc = std::min(nt.minc, q);
        }
      const int id = (int)T.size();
      T.push_back(nt);
      for (int k = 0; k < 4; ++k)
        if (k != apex && nt.v[k] != kInf) entries.push_back({nt.v[k], p});
      next.push_back({id, ts});
      for (int k = 0; k < 4; ++k) {
        if (k == apex) continue;
        int f[3], m = 0;
        for (int l = 0; l < 4; ++l)
          if (l != k) f[m++] = nt.v[l];
        const uint64_t key = ridge_key(f[0], f[1], f[2]);
        auto it = waiting.find(key);
        if (it == waiting.end()) {
          waiting[key] = id;
        } else {
          next.push_back({id, it->second});
          waiting.erase(it);
        }
      }
    }
    items.swap(next);
  }
  std::sort(entries.begin(), entries.end());
  entries.erase(std::unique(entries.begin(), entries.end()), entries.end());
  size_t e = 0;
  for (int i = 0; i < n; ++i)
    for (int64_t x = ref.off[i]; x < ref.off[i + 1]; ++x, ++e)
      if (e >= entries.size() || entries[e].first != i || entries[e].second != ref.ent[x]) {
        printf("list %d differs at entry %lld\n", i, (long long)(x - ref.off[i]));
        return 1;
      }
  if (e != entries.size()) {
    printf("%zu extra entries\n", entries.size() - e);
    return 1;
  }
  if (!waiting.empty()) {
    printf("%zu ridges left with one tetrahedron\n", waiting.size());
    return 1;
  }
  printf("ok rounds=%d tets=%zu entries=%zu\n", rounds, T.size(), e);
  return 0;
}
