// Internal definition of a cloud handle, shared by the host and device translation units.
#pragma once
#include <atomic>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "delaunay.h"
#include "mknn.h"

namespace mknn {
// Successor (or predecessor) lists that can be edited in place: list r occupies
// pool[start[r] .. start[r] + len[r]), ascending, with room for cap[r] entries; a list that
// outgrows its room moves to the end of the pool.
struct DynLists {
  std::vector<int64_t> start;
  std::vector<int32_t> len, cap;
  std::vector<int32_t> pool;

  void from_csr(const Csr &c, int64_t n);
  void to_csr(Csr *c, int64_t n) const;
  const int32_t *begin(int64_t r) const { return pool.data() + start[r]; }
  int32_t size(int64_t r) const { return len[r]; }
  bool contains(int64_t r, int32_t v) const;
  void insert_sorted(int64_t r, int32_t v);
  bool erase(int64_t r, int32_t v);
  void clear(int64_t r) { len[r] = 0; }
  void grow(int64_t n) {   // new, empty lists up to n
    start.resize(n, 0);
    len.resize(n, 0);
    cap.resize(n, 0);
  }
};

// The triangulation of the live sites kept for appending points (insertion), built at the
// first insertion; deletions remove their sites from it.
struct InsertState {
  std::vector<double> P;                       // all sites by rank, float64
  std::unique_ptr<DelaunayBuilder> dt;         // live sites inserted in rank order
};
// List segments rewritten by a deletion batch, ready to be appended to the device arena.
// The whole device image of the lists: records {x, y, z, rank bits} of every list, lists in
// the Morton order of their owners, then padding; one {start, length} descriptor per rank.
struct HostPack {
  std::vector<float> ent;          // 4 floats per record
  std::vector<uint64_t> lst;
  std::vector<float> pts;          // 4 floats per rank {x, y, z, 0}
  int64_t nnz = 0;                 // records in use
  int64_t cap = 0;                 // records to allocate (slack for later deltas + padding)
};
// List segments rewritten by a deletion batch, ready to be appended to the device arena, or,
// when the arena's slack would run out, a complete new image of the lists.
struct DeviceDelta {
  bool on_device = false;
  std::vector<int32_t> ranks;      // lists that changed
  std::vector<uint32_t> lens;      // their new lengths
  std::vector<float> rec;          // their new records {x, y, z, rank bits}, concatenated
  std::vector<uint64_t> desc;      // new descriptors (filled when applied)
  std::vector<float> new_pts;      // appended points {x, y, z, 0}, ranks pts_from ..
  int64_t pts_from = 0;
  bool repack = false;             // apply `pack` as a new arena instead
  HostPack pack;
  void *old_ent = nullptr;         // arena replaced by a re-pack: free once its readers are done
  uint64_t *old_lst = nullptr;
  void *old_pts = nullptr;
};
}  // namespace mknn

struct mknn_cloud {
  std::atomic<int64_t> n{0};       // ranks so far (atomic: a server's clients read it while a
                                   // worker appends points)
  std::vector<float> xyz;          // n x 3 float32 by rank
  std::vector<int32_t> order;      // rank -> caller id
  mknn::Csr succ;                  // successor lists (ranks ascending)
  mknn::Csr pred;                  // Delaunay neighbours at insertion (transpose of succ)
  std::vector<uint8_t> live;       // 1 = present
  bool editable = false;           // dsucc/dpred hold the lists (after the first deletion)
  bool csr_dirty = false;          // succ/pred CSR views are stale
  mknn::DynLists dsucc, dpred;
  int32_t head = 0;                // smallest live rank
  int64_t nlive = 0;
  float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};   // bounding box of all points
  std::unique_ptr<mknn::InsertState> ins;      // see InsertState
  // Bumped by every mutation of the host lists.  A deletion on an uploaded cloud bumps it
  // only when its device delta is applied, so the device copy stays usable (on the old
  // lists) while the host part of the deletion runs on another thread.
  std::atomic<uint64_t> version{0};

  // device residency
  int device = -1;
  void *d_ent = nullptr;           // 16-byte records {x, y, z, rank}, padded
  uint64_t *d_lst = nullptr;       // per rank: start | (length << 32)
  void *d_pts = nullptr;           // per rank: {x, y, z, 0} (for statistics of k-NN rows)
  int64_t ent_used = 0, ent_cap = 0;   // records in use / allocated (slack takes deltas)
  int64_t lst_cap = 0;             // descriptors allocated (slack for appended points)
  int64_t dev_bytes = 0;
  std::atomic<uint64_t> dev_version{~0ull};
  // What the device lists describe, recorded when they were installed or last updated:
  // query launches read these, never the host fields above, which a worker thread of a
  // server may be changing for the next update batch.
  int32_t dev_head = 0;            // the head of the lists on the device
  float dev_hxyz[3] = {0, 0, 0};   // its coordinates
  int64_t dev_n = 0;               // ranks the device lists cover
  float dev_lo[3] = {0, 0, 0}, dev_hi[3] = {0, 0, 0};   // bounding box (for query bucketing)

  // Pending (lazy) deletions: ranks marked as deleted that the device lists still hold
  // until Alg. 3 is applied to them.  The device array holds, per rank, the epoch of the
  // batch that marked it (0: never marked); an entry keeps its epoch after its deletion is
  // applied (the rank is then in no list).  mknn_delete_lazy marks in epochs
  // lazy_epoch + 1, ...; a server marks in epochs of its own.
  std::vector<int32_t> lazy;       // mknn_delete_lazy: pending ranks, in arrival order
  std::vector<uint8_t> lazy_mark;  // per rank: 1 = pending
  uint32_t lazy_epoch = 0;         // the last epoch mknn_delete_lazy marked in
  uint32_t *d_dead = nullptr;      // device epochs, dead_cap entries
  int64_t dead_cap = 0;
  uint32_t *d_overflow = nullptr;  // device counter of rows a lazy launch could not certify
  std::atomic<int64_t> dev_lazy{0};   // marked ranks that launches must filter (0: none)
};

namespace mknn {
mknn_status set_error(mknn_status s, const std::string &msg);
void clear_error();
// Deletes ranks[0..count) from the host lists (Alg. 3).  On success, *changed receives
// every rank whose successor list changed (for the device update).
mknn_status delete_ranks_host(mknn_cloud *c, const int32_t *ranks, int64_t count,
                              std::vector<int32_t> *changed);
// Appends xyz[0..count) (float32 [count][3]) as ranks n .. n+count-1 (Sec. 3 insertion):
// every live Delaunay neighbour of a new site gets its rank appended.  On success *changed
// receives every rank whose list changed or is new.
mknn_status insert_points_host(mknn_cloud *c, const float *xyz, int64_t count,
                               std::vector<int32_t> *changed);
void refresh_csr(mknn_cloud *c);
}  // namespace mknn
