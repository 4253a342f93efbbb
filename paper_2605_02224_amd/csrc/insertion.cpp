// Point insertion: appending sites to the birth order (Sec. 3 construction, continued).
//
// A new site p gets the next rank r = n.  Its successor list is empty (no site is younger),
// and r is appended to the list of every Delaunay neighbour of p in the triangulation of the
// live sites plus p -- exactly what the construction would have done had p been inserted
// last.  Lists stay ascending because r is the largest rank.
//
// The triangulation of the live sites is built (in rank order) at the first insertion and
// kept.  A deletion removes its sites from it as well (the star of a removed vertex is
// refilled from the triangulation of its link); should that fail, it is dropped and the next
// insertion triangulates the live sites again.  Either way it records the same lists the
// cloud holds: the lists after a deletion equal those of the remaining sites inserted in
// the original relative order.
#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <tuple>

#include "cloud.h"
#include "delaunay.h"

namespace mknn {

mknn_status insert_points_host(mknn_cloud *c, const float *xyz, int64_t count,
                               std::vector<int32_t> *changed) {
  if (count < 1) return MKNN_OK;
  if (c->n + count > ((int64_t)1 << 30))
    return set_error(MKNN_EUNSUPPORTED, "mknn_insert: more than 2^30 points");
  if (c->nlive < 4)
    return set_error(MKNN_EUNSUPPORTED, "mknn_insert: needs at least four live points");
  // validate the whole batch before touching anything
  std::vector<std::tuple<float, float, float, int64_t>> key((size_t)count);
  for (int64_t t = 0; t < count; ++t) {
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(xyz[3 * t + k]))
        return set_error(MKNN_ENONFINITE, "mknn_insert: non-finite coordinate at point " +
                                              std::to_string(t));
    key[t] = std::make_tuple(xyz[3 * t], xyz[3 * t + 1], xyz[3 * t + 2], t);
  }
  std::sort(key.begin(), key.end());
  for (int64_t t = 1; t < count; ++t)
    if (std::get<0>(key[t]) == std::get<0>(key[t - 1]) &&
        std::get<1>(key[t]) == std::get<1>(key[t - 1]) &&
        std::get<2>(key[t]) == std::get<2>(key[t - 1]))
      return set_error(MKNN_EDUPLICATE, "mknn_insert: points " + std::to_string(std::get<3>(key[t - 1])) +
                                            " and " + std::to_string(std::get<3>(key[t])) +
                                            " coincide");
  try {
    if (!c->ins) {
      auto st = std::make_unique<InsertState>();
      st->P.assign(c->xyz.begin(), c->xyz.end());
      st->dt = std::make_unique<DelaunayBuilder>(st->P.data(), c->n);
      std::vector<int32_t> order;
      order.reserve((size_t)c->nlive);
      for (int64_t r = 0; r < c->n; ++r)
        if (c->live[r]) order.push_back((int32_t)r);
      st->dt->set_order(std::move(order));
      int64_t bad = -1;
      const BuildStatus bs = st->dt->build(&bad);
      if (bs != kBuildOk)
        return set_error(MKNN_EUNSUPPORTED,
                         bs == kBuildDegenerateStart
                             ? "mknn_insert: the four oldest live points are coplanar"
                             : "mknn_insert: triangulating the live points failed at rank " +
                                   std::to_string(bad));
      c->ins = std::move(st);
    }
    InsertState &S = *c->ins;
    for (int64_t t = 0; t < count; ++t) {
      double p[3] = {xyz[3 * t], xyz[3 * t + 1], xyz[3 * t + 2]};
      double d = 0;
      S.dt->nearest(p, &d);
      if (d == 0.0)
        return set_error(MKNN_EDUPLICATE, "mknn_insert: point " + std::to_string(t) +
                                              " coincides with a live point");
    }
    // append: coordinates, triangulation, lists
    if (!c->editable) {
      c->dsucc.from_csr(c->succ, c->n);
      c->dpred.from_csr(c->pred, c->n);
      c->editable = true;
    }
    const int64_t n0 = c->n, n1 = c->n + count;
    c->xyz.insert(c->xyz.end(), xyz, xyz + 3 * count);
    S.P.insert(S.P.end(), c->xyz.begin() + 3 * n0, c->xyz.end());
    S.dt->grow(S.P.data(), n1);
    c->dsucc.grow(n1);
    c->dpred.grow(n1);
    std::vector<char> mark((size_t)n1, 0);
    for (int64_t t = 0; t < count; ++t) {
      const int32_t r = (int32_t)(n0 + t);
      const BuildStatus bs = S.dt->insert_next();
      if (bs != kBuildOk) {
        // the earlier points of the batch are in: keep them, drop the rest
        c->xyz.resize(3 * (size_t)r);
        c->ins.reset();
        c->n = r;
        c->dsucc.grow(r);
        c->dpred.grow(r);
        c->csr_dirty = true;
        ++c->version;
        return set_error(MKNN_EUNSUPPORTED, "mknn_insert: inserting point " + std::to_string(t) +
                                                " failed");
      }
      for (int32_t i : S.dt->last_neighbors()) {
        c->dsucc.insert_sorted(i, r);
        c->dpred.insert_sorted(r, i);
        if (!mark[i]) {
          mark[i] = 1;
          changed->push_back(i);
        }
      }
      mark[r] = 1;
      changed->push_back(r);
      c->live.push_back(1);
      c->order.push_back((int32_t)r);
      ++c->nlive;
      for (int k = 0; k < 3; ++k) {   // the bounding box covers every point inserted
        c->lo[k] = std::min(c->lo[k], c->xyz[3 * (int64_t)r + k]);
        c->hi[k] = std::max(c->hi[k], c->xyz[3 * (int64_t)r + k]);
      }
      c->n = r + 1;
    }
    c->csr_dirty = true;
  } catch (const std::bad_alloc &) {
    c->ins.reset();
    return set_error(MKNN_ENOMEM, "mknn_insert: out of host memory");
  }
  return MKNN_OK;
}

}  // namespace mknn
