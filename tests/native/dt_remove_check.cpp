// Checks vertex removal of the host triangulation against triangulating the remaining
// sites from scratch: same tetrahedra (as vertex sets, ghosts included), a valid structure,
// and empty circumspheres.  Usage: dt_remove_check <n> <removals> <seed> <shape>
// (shape 0: uniform cube, 1: sphere shell, 2: integer grid with jitter-free cospherical
// quadruples).  Prints "ok <removed> <tets>" or the first mismatch; exit status 0 on ok.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "delaunay.h"

using mknn::DelaunayBuilder;

static std::set<std::vector<int>> tets_of(const DelaunayBuilder &dt, const std::vector<int> &map);

int main(int argc, char **argv) {
  if (argc < 5) return 2;
  const int n = atoi(argv[1]), nrem = atoi(argv[2]), seed = atoi(argv[3]), shape = atoi(argv[4]);
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> P(3 * n);
  for (int i = 0; i < n; ++i) {
    double x = U(rng), y = U(rng), z = U(rng);
    if (shape == 1) {
      const double r = std::sqrt(x * x + y * y + z * z) + 1e-300;
      x /= r; y /= r; z /= r;
    } else if (shape == 2) {
      x = std::floor(4 * (x + 1)); y = std::floor(4 * (y + 1)); z = std::floor(4 * (z + 1));
    }
    P[3 * i] = (float)x; P[3 * i + 1] = (float)y; P[3 * i + 2] = (float)z;
  }
  // drop exact duplicates (the grid shape makes many), keeping the first
  std::vector<int> keep;
  {
    std::set<std::vector<double>> seen;
    for (int i = 0; i < n; ++i)
      if (seen.insert({P[3 * i], P[3 * i + 1], P[3 * i + 2]}).second) keep.push_back(i);
  }
  std::vector<double> Q(3 * keep.size());
  for (size_t a = 0; a < keep.size(); ++a)
    for (int d = 0; d < 3; ++d) Q[3 * a + d] = P[3 * keep[a] + d];
  const int m = (int)keep.size();
  DelaunayBuilder dt(Q.data(), m);
  int64_t bad = -1;
  if (dt.build(&bad) != mknn::kBuildOk) { printf("build failed\n"); return 1; }
  std::vector<char> alive(m, 1);
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::shuffle(order.begin(), order.end(), rng);
  int removed = 0, refused = 0;
  for (int t = 0; t < nrem && t < m - 5; ++t) {
    const int v = order[t];
    const mknn::BuildStatus st = dt.remove(v);
    if (st != mknn::kBuildOk) { ++refused; continue; }
    alive[v] = 0;
    ++removed;
    std::string why;
    if (!dt.validate(&why)) { printf("invalid after removing %d: %s\n", v, why.c_str()); return 1; }
  }
  std::string why;
  if (m <= 400 && !dt.validate_empty_spheres(&why)) { printf("spheres: %s\n", why.c_str()); return 1; }
  // reference: the remaining sites triangulated from scratch, in id order
  std::vector<int> ids;
  for (int i = 0; i < m; ++i) if (alive[i]) ids.push_back(i);
  std::vector<double> R(3 * ids.size());
  for (size_t a = 0; a < ids.size(); ++a)
    for (int d = 0; d < 3; ++d) R[3 * a + d] = Q[3 * ids[a] + d];
  DelaunayBuilder ref(R.data(), (int64_t)ids.size());
  if (ref.build(&bad) != mknn::kBuildOk) { printf("reference build failed\n"); return 1; }
  std::vector<int> ident(m);
  for (int i = 0; i < m; ++i) ident[i] = i;
  const auto a = tets_of(dt, ident), b = tets_of(ref, ids);
  if (a != b) {
    printf("tetrahedra differ: %zu vs %zu\n", a.size(), b.size());
    return 1;
  }
  printf("ok %d %zu refused %d\n", removed, a.size(), refused);
  return refused ? 3 : 0;
}

// every tetrahedron as its sorted vertex ids (mapped), ghosts with -1
static std::set<std::vector<int>> tets_of(const DelaunayBuilder &dt, const std::vector<int> &map) {
  std::set<std::vector<int>> out;
  for (int64_t t = 0; t < dt.num_tet_slots(); ++t) {
    int v[4];
    if (!dt.tet(t, v)) continue;
    std::vector<int> k(4);
    for (int i = 0; i < 4; ++i) k[i] = v[i] < 0 ? -1 : map[v[i]];
    std::sort(k.begin(), k.end());
    out.insert(k);
  }
  return out;
}
