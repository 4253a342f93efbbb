// Site deletion by local Delaunay updates (Sec. 4.3, Alg. 3, Lemmas 1 and 2).
//
// Deleting p_i must leave the successor lists equal to those of P \ {p_i} inserted in the
// original relative order.  Lemma 1: an entry not involving p_i stays valid.  So the work is
//   pruning       -- remove i from every list that holds it (the lists of pred[i], the
//                    Delaunay neighbours of p_i at its insertion), and drop L_i;
//   redistribution -- find the adjacencies that appear once p_i is gone.  By Lemma 2, a pair
//                    (p_j, p_k), j < k, that becomes adjacent at time k consists of two
//                    Voronoi neighbours of p_i at time k, i.e. members of
//                    Loc_k = pred[i] + {entries of L_i up to k}, and k itself is in L_i.
//
// For every k in L_i, in order, p_k is inserted into the Delaunay triangulation of Loc_k (the
// local set without p_i, built incrementally in rank order); every Delaunay neighbour p_j of
// p_k that is not already adjacent (k not in L_j) is a candidate.  Acceptance (the garbled
// quantifier of Alg. 3 read as "some shared Voronoi vertex lies strictly inside the old
// cell of p_i"): the pair is accepted iff some tetrahedron of the local triangulation around
// edge (j, k) -- a Voronoi vertex of their shared facet, ghosts included for unbounded facets
// -- has p_i strictly inside its circumsphere.  Inside the old cell of p_i the nearest sites
// of P \ {p_i} are neighbours of p_i, all in Loc_k, so the local facet agrees there with the
// global one, and by Lemma 2 a new facet lies wholly inside that cell: the test is exact.
//
// While Loc_k holds at most three points (only possible for the three oldest ranks), Loc_k is
// the whole prefix P_{1:k} \ {p_i} and adjacency is decided directly: two or three sites are
// pairwise adjacent, except that the middle of three collinear sites separates the other two.
//
// A batch is reordered into rounds of independent deletions.  The lists after deleting a set
// are those of the remaining points (Sec. 4.3), whatever the order, and the work for p_i
// reads only the lists of i and of its local set Loc(i) = pred[i] + L_i and writes only
// theirs; so deletions whose closed local sets {i} + Loc(i) are pairwise disjoint see the
// same lists in any order.  Each round takes, in batch order, every remaining deletion whose
// closed local set meets none already taken; the redistributions of a round run on several
// threads, and their edits are then applied in batch order.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "cloud.h"
#include "delaunay.h"
#include "exact.h"

namespace mknn {

void DynLists::from_csr(const Csr &c, int64_t n) {
  start.resize(n);
  len.resize(n);
  cap.resize(n);
  pool.clear();
  pool.reserve(c.ent.size() + (size_t)n * 2);
  for (int64_t r = 0; r < n; ++r) {
    const int32_t l = (int32_t)(c.off[r + 1] - c.off[r]);
    start[r] = (int64_t)pool.size();
    len[r] = l;
    cap[r] = l + 2;
    pool.insert(pool.end(), c.ent.begin() + c.off[r], c.ent.begin() + c.off[r + 1]);
    pool.push_back(0);
    pool.push_back(0);
  }
}

void DynLists::to_csr(Csr *c, int64_t n) const {
  c->off.assign(n + 1, 0);
  for (int64_t r = 0; r < n; ++r) c->off[r + 1] = c->off[r] + len[r];
  c->ent.resize(c->off[n]);
  for (int64_t r = 0; r < n; ++r)
    if (len[r]) std::memcpy(&c->ent[c->off[r]], begin(r), sizeof(int32_t) * len[r]);
}

bool DynLists::contains(int64_t r, int32_t v) const {
  const int32_t *b = begin(r);
  return std::binary_search(b, b + len[r], v);
}

void DynLists::insert_sorted(int64_t r, int32_t v) {
  if (len[r] == cap[r]) {
    const int32_t nc = std::max(8, 2 * cap[r]);
    const int64_t ns = (int64_t)pool.size();
    pool.resize(pool.size() + nc);
    if (len[r]) std::memmove(&pool[ns], &pool[start[r]], sizeof(int32_t) * len[r]);
    start[r] = ns;
    cap[r] = nc;
  }
  int32_t *b = pool.data() + start[r];
  int32_t *pos = std::lower_bound(b, b + len[r], v);
  if (pos != b + len[r] && *pos == v) return;
  std::memmove(pos + 1, pos, sizeof(int32_t) * (size_t)(b + len[r] - pos));
  *pos = v;
  ++len[r];
}

bool DynLists::erase(int64_t r, int32_t v) {
  int32_t *b = pool.data() + start[r];
  int32_t *pos = std::lower_bound(b, b + len[r], v);
  if (pos == b + len[r] || *pos != v) return false;
  std::memmove(pos, pos + 1, sizeof(int32_t) * (size_t)(b + len[r] - pos - 1));
  --len[r];
  return true;
}

void refresh_csr(mknn_cloud *c) {
  if (!c->editable || !c->csr_dirty) return;
  c->dsucc.to_csr(&c->succ, c->n);
  c->dpred.to_csr(&c->pred, c->n);
  c->csr_dirty = false;
}

namespace {

// Adjacency among at most three sites (the whole prefix): see the file comment.
bool tiny_adjacent(const std::vector<const double *> &pts, int a, int b) {
  if (pts.size() <= 2) return true;
  const int m = 3 - a - b;   // the third site (indices 0, 1, 2)
  const double *pa = pts[a], *pb = pts[b], *pm = pts[m];
  bool collinear = true;
  for (int k = 0; k < 3; ++k) collinear &= cross_component_sign(pa, pb, pm, k) == 0;
  if (!collinear) return true;
  Expansion s;   // m strictly between a and b: (a - m).(b - m) < 0
  for (int k = 0; k < 3; ++k) s = add(s, mul(diff(pa[k], pm[k]), diff(pb[k], pm[k])));
  return !(s.sign() < 0);
}

struct NewEntry {
  int32_t owner, rank;
};

// Redistribution for one deleted rank; fills `adds` with the new (owner, rank) entries.
mknn_status redistribute(mknn_cloud *c, int32_t i, std::vector<NewEntry> *adds) {
  const float *P = c->xyz.data();
  std::vector<int32_t> loc;   // local set by ascending rank: pred[i] then L_i
  const int32_t np = c->dpred.size(i), ns = c->dsucc.size(i);
  loc.insert(loc.end(), c->dpred.begin(i), c->dpred.begin(i) + np);
  loc.insert(loc.end(), c->dsucc.begin(i), c->dsucc.begin(i) + ns);
  const int64_t L = (int64_t)loc.size();
  if (ns == 0) return MKNN_OK;
  std::vector<double> lp(3 * L);
  for (int64_t t = 0; t < L; ++t)
    for (int d = 0; d < 3; ++d) lp[3 * t + d] = (double)P[3 * (int64_t)loc[t] + d];
  double pi_xyz[3];
  for (int d = 0; d < 3; ++d) pi_xyz[d] = (double)P[3 * (int64_t)i + d];
  const double *pi = pi_xyz;
  DelaunayBuilder dt(lp.data(), L);
  int64_t inserted = 0;   // local ids inserted into dt
  for (int64_t t = np; t < L; ++t) {
    const int32_t k = loc[t];
    const int64_t cnt = t + 1;   // |Loc_k|
    if (cnt <= 3) {
      std::vector<const double *> pts;
      for (int64_t u = 0; u < cnt; ++u) pts.push_back(&lp[3 * u]);
      for (int64_t u = 0; u < t; ++u) {
        const int32_t j = loc[u];
        if (!c->dsucc.contains(j, k) && tiny_adjacent(pts, (int)u, (int)t))
          adds->push_back({j, k});
      }
      continue;
    }
    while (inserted < cnt) {
      const BuildStatus st = dt.insert_next();
      if (st == kBuildDegenerateStart)
        return set_error(MKNN_EUNSUPPORTED,
                         "mknn_delete: the oldest four sites around rank " + std::to_string(i) +
                             " are coplanar; the local triangulation cannot start");
      if (st != kBuildOk)
        return set_error(MKNN_EUNSUPPORTED, "mknn_delete: local triangulation failed around rank " +
                                                std::to_string(i));
      inserted = dt.inserted();
    }
    for (int32_t uj : dt.last_neighbors()) {
      const int32_t j = loc[uj];
      if (c->dsucc.contains(j, k)) continue;          // already adjacent before deletion
      if (dt.edge_in_conflict(uj, (int32_t)t, pi)) adds->push_back({j, k});
    }
  }
  return MKNN_OK;
}

// Helper threads for the redistributions, shared by every deletion in the process: at most
// the CPU budget (OMP_NUM_THREADS when set, else the hardware threads) minus one per caller.
std::atomic<int> g_helpers{-1};

int cpu_budget() {
  const char *e = std::getenv("OMP_NUM_THREADS");
  int v = e ? std::atoi(e) : 0;
  if (v <= 0) v = (int)std::thread::hardware_concurrency();
  return std::max(1, v);
}

int take_helpers(int want) {
  int cur = g_helpers.load();
  if (cur < 0) {
    int init = -1;
    g_helpers.compare_exchange_strong(init, cpu_budget() - 1);
    cur = g_helpers.load();
  }
  while (want > 0 && cur > 0) {
    const int got = std::min(want, cur);
    if (g_helpers.compare_exchange_weak(cur, cur - got)) return got;
  }
  return 0;
}

void give_helpers(int n) { if (n > 0) g_helpers.fetch_add(n); }

struct RoundItem {
  int32_t rank;
  std::vector<NewEntry> adds;
  mknn_status st = MKNN_OK;
  std::string err;
};

// Redistributions of one round, on the calling thread and up to `helpers` more.
void run_round(mknn_cloud *c, std::vector<RoundItem> &items, int helpers) {
  std::atomic<size_t> next{0};
  auto work = [&]() {
    for (;;) {
      const size_t t = next.fetch_add(1);
      if (t >= items.size()) return;
      RoundItem &it = items[t];
      try {
        it.st = redistribute(c, it.rank, &it.adds);
        if (it.st != MKNN_OK) it.err = mknn_last_error();
      } catch (const std::bad_alloc &) {
        it.st = MKNN_ENOMEM;
        it.err = "mknn_delete: out of host memory";
      }
    }
  };
  std::vector<std::thread> th;
  const int nh = std::min<int>(helpers, (int)items.size() - 1);
  for (int h = 0; h < nh; ++h) th.emplace_back(work);
  work();
  for (std::thread &t : th) t.join();
}

}  // namespace

mknn_status delete_ranks_host(mknn_cloud *c, const int32_t *ranks, int64_t count,
                              std::vector<int32_t> *changed) {
  // validate the whole batch before touching anything
  std::vector<int32_t> del(ranks, ranks + count);
  std::vector<int32_t> sorted = del;
  std::sort(sorted.begin(), sorted.end());
  for (size_t t = 0; t < sorted.size(); ++t) {
    const int32_t r = sorted[t];
    if (r < 0 || r >= c->n || !c->live[r])
      return set_error(MKNN_ENOTFOUND, "mknn_delete: rank " + std::to_string(r) +
                                           " is unknown or already deleted");
    if (t && sorted[t - 1] == r)
      return set_error(MKNN_ENOTFOUND, "mknn_delete: rank " + std::to_string(r) +
                                           " appears twice in the batch");
  }
  if (c->nlive - count < 1)
    return set_error(MKNN_EINVAL, "mknn_delete: a cloud must keep at least one point");
  try {
    if (!c->editable) {
      c->dsucc.from_csr(c->succ, c->n);
      c->dpred.from_csr(c->pred, c->n);
      c->editable = true;
    }
    std::vector<char> mark(c->n, 0);
    std::vector<uint32_t> claim(c->n, 0);   // round stamp of the ranks a round's work touches
    uint32_t round = 0;
    bool applied_any = false;
    std::vector<int32_t> rest = del, later;
    std::vector<RoundItem> items;
    while (!rest.empty()) {
      // ---- one round: every remaining deletion whose closed local set is still free
      ++round;
      items.clear();
      later.clear();
      for (int32_t i : rest) {
        const int32_t *pb = c->dpred.begin(i), *sb = c->dsucc.begin(i);
        const int32_t np = c->dpred.size(i), ns = c->dsucc.size(i);
        bool free = claim[i] != round;
        for (int32_t t = 0; free && t < np; ++t) free = claim[pb[t]] != round;
        for (int32_t t = 0; free && t < ns; ++t) free = claim[sb[t]] != round;
        if (!free) {
          later.push_back(i);
          continue;
        }
        claim[i] = round;
        for (int32_t t = 0; t < np; ++t) claim[pb[t]] = round;
        for (int32_t t = 0; t < ns; ++t) claim[sb[t]] = round;
        items.emplace_back();
        items.back().rank = i;
      }
      const int helpers = items.size() > 1 ? take_helpers((int)items.size() - 1) : 0;
      run_round(c, items, helpers);
      give_helpers(helpers);
      // ---- apply the round's edits in batch order
      for (RoundItem &it : items) {
        const int32_t i = it.rank;
        if (it.st != MKNN_OK) {
          c->ins.reset();
          if (applied_any) {
            // ranks applied before this one stay deleted: the host lists have moved on,
            // and a device copy stays stale until the next upload
            c->csr_dirty = true;
            ++c->version;
          }
          return set_error(it.st, it.err);
        }
        for (const NewEntry &e : it.adds) {
          c->dsucc.insert_sorted(e.owner, e.rank);
          c->dpred.insert_sorted(e.rank, e.owner);
          if (!mark[e.owner]) { mark[e.owner] = 1; changed->push_back(e.owner); }
        }
        // pruning
        for (int32_t t = 0; t < c->dpred.size(i); ++t) {
          const int32_t j = c->dpred.begin(i)[t];
          c->dsucc.erase(j, i);
          if (!mark[j]) { mark[j] = 1; changed->push_back(j); }
        }
        for (int32_t t = 0; t < c->dsucc.size(i); ++t) c->dpred.erase(c->dsucc.begin(i)[t], i);
        c->dsucc.clear(i);
        c->dpred.clear(i);
        if (!mark[i]) { mark[i] = 1; changed->push_back(i); }
        c->live[i] = 0;
        --c->nlive;
        if (i == c->head) {
          int32_t h = i + 1;
          while (h < c->n && !c->live[h]) ++h;
          c->head = h;
        }
        applied_any = true;
      }
      rest.swap(later);
    }
    c->csr_dirty = true;
    if (c->ins) {
      // the triangulation kept for insertion loses the deleted sites too, and the lists its
      // point location walks follow the cloud's; a removal it cannot do drops it (the next
      // insertion triangulates the live sites again)
      DelaunayBuilder &dt = *c->ins->dt;
      for (int32_t i : del)
        if (dt.remove(i) != kBuildOk) {
          c->ins.reset();
          break;
        }
      if (c->ins)
        for (int32_t r : *changed) dt.set_list(r, c->dsucc.begin(r), c->dsucc.size(r));
    }
  } catch (const std::bad_alloc &) {
    c->ins.reset();
    c->csr_dirty = true;
    ++c->version;   // possibly half-applied: treat every device copy as stale
    return set_error(MKNN_ENOMEM, "mknn_delete: out of host memory");
  }
  return MKNN_OK;
}

}  // namespace mknn
