// Device half of the C ABI: residency of successor lists in HBM, query batch preparation,
// the query kernels and their launch configuration (with the autotuner's table), list
// deltas for deletion and insertion, and the plane fit.
//
// Three kernel families compute the same rows (the 1-NN descent of Alg. 1, the k-expansion
// of Alg. 2, the prefix bound of Sec. 4.2), with identical float64 keys (D, rank):
//   lane  (knn_lane_kernel, below): one query per lane, N a register-resident sorted array;
//   group (knn_group.h): 16 lanes per query, the four rows of a wavefront in lockstep phases
//         (it also carries the work-counting variant);
//   rows  (knn_rows.h): 16 lanes per query, rows scheduled independently -- the default.
// In the lane kernel every examined entry, transition sites included, is offered to N;
// offering more true sites than Alg. 1 does never changes the result, and it lets the
// final, completely scanned list of the descent serve as Alg. 2's first iteration.
// Distances are evaluated in float64 exactly as the brute-force definition (each operation
// rounded, no FMA), so ties resolve identically.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <new>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "device_common.h"
#include "knn_group.h"
#include "knn_rows.h"
#include "planefit.h"

namespace mknn {

template <int K>
struct TopK {
  double d[K];
  int32_t r[K];
  double thr_d;
  int32_t thr_r;

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      d[j] = INFINITY;
      r[j] = kEmpty;
    }
    thr_d = INFINITY;
    thr_r = kEmpty;
  }

  // Key of the candidate that follows the last expanded one: the first slot whose key is
  // greater than (ld, lr).  A compare chain, not an index, so N stays in registers.
  __device__ __forceinline__ void next_after(double &ld, int32_t &lr) const {
    int32_t v = kEmpty;
    double vd = INFINITY;
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
      bool gt = d[j] > ld || (d[j] == ld && r[j] > lr);
      v = gt ? r[j] : v;
      vd = gt ? d[j] : vd;
    }
    ld = vd;
    lr = v;
  }

  template <bool EXACTK>
  __device__ __forceinline__ int insert(double dd, int32_t rr, int k) {
    if (!(dd < thr_d || (dd == thr_d && rr < thr_r))) return 0;
    bool dup = false;
#pragma unroll
    for (int j = 0; j < K; ++j) dup |= (r[j] == rr);
    if (dup) return 0;
    // replace the last slot, then bubble the candidate towards the front
    d[K - 1] = dd;
    r[K - 1] = rr;
#pragma unroll
    for (int j = K - 1; j >= 1; --j) {
      bool sw = d[j] < d[j - 1] || (d[j] == d[j - 1] && r[j] < r[j - 1]);
      double td = d[j - 1];
      int32_t tr = r[j - 1];
      d[j - 1] = sw ? d[j] : td;
      r[j - 1] = sw ? r[j] : tr;
      d[j] = sw ? td : d[j];
      r[j] = sw ? tr : r[j];
    }
    if (EXACTK) {
      thr_d = d[K - 1];
      thr_r = r[K - 1];
    } else {
      double td = d[0];
      int32_t tr = r[0];
#pragma unroll
      for (int j = 1; j < K; ++j) {
        td = (j == k - 1) ? d[j] : td;
        tr = (j == k - 1) ? r[j] : tr;
      }
      thr_d = td;
      thr_r = tr;
    }
    return 1;
  }
};

// One query per lane.  K = register capacity (>= k); EXACTK: k == K for every query.
template <int K, bool EXACTK, bool COUNT>
__global__ __launch_bounds__(256) void knn_lane_kernel(QueryArgs a) {
  const int64_t s = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (s >= a.nq) return;
  double qx, qy, qz;
  int64_t qi;
  if (a.qs) {
    float4 v = a.qs[s];
    qx = v.x;
    qy = v.y;
    qz = v.z;
    qi = __float_as_int(v.w);
  } else {
    qi = s;
    qx = a.q[3 * s];
    qy = a.q[3 * s + 1];
    qz = a.q[3 * s + 2];
  }
  const int k = a.kq ? a.kq[qi] : a.k;
  int64_t mm = a.mq ? (int64_t)a.mq[qi] : (int64_t)a.m;
  if (mm > a.n) mm = a.n;
  const int32_t m = (int32_t)mm;
  const int64_t row = a.row_off ? a.row_off[qi] : qi * (int64_t)a.k;
  if (k < 1 || k > K || m < 1) return;

  TopK<K> N;
  N.init();
  int32_t nent = 0, nlist = 0, nins = 0;

  if (a.head < m) {
    // ---- Alg. 1: descent from the head, every examined entry inserted into N
    int32_t cur = a.head;
    double dcur = sq_dist(qx, qy, qz, make_float4(a.hx, a.hy, a.hz, 0.f));
    nins += N.template insert<EXACTK>(dcur, cur, k);
    for (;;) {
      const uint64_t dsc = a.lst[cur];
      const uint32_t st = (uint32_t)dsc, len = (uint32_t)(dsc >> 32);
      if (COUNT) ++nlist;
      bool jumped = false;
      float4 nx = a.ent[st];
      for (uint32_t e = 0; e < len; ++e) {
        const float4 c = nx;
        nx = a.ent[st + e + 1];
        const int32_t r = __float_as_int(c.w);
        if (r >= m) break;
        const double dd = sq_dist(qx, qy, qz, c);
        if (COUNT) ++nent;
        nins += N.template insert<EXACTK>(dd, r, k);
        if (dd < dcur) {
          cur = r;
          dcur = dd;
          jumped = true;
          break;
        }
      }
      if (!jumped) break;
    }
    // ---- Alg. 2: expand the lists of the confirmed neighbours N[2..k-1] (1-based)
    double ld = N.d[0];
    int32_t lr = N.r[0];
    for (int i = 1; i < k - 1; ++i) {
      N.next_after(ld, lr);
      const int32_t pr = lr;
      if (pr == kEmpty) break;
      const uint64_t dsc = a.lst[pr];
      const uint32_t st = (uint32_t)dsc, len = (uint32_t)(dsc >> 32);
      if (COUNT) ++nlist;
      float4 nx = a.ent[st];
      for (uint32_t e = 0; e < len; ++e) {
        const float4 c = nx;
        nx = a.ent[st + e + 1];
        const int32_t r = __float_as_int(c.w);
        if (r >= m) break;
        if (COUNT) ++nent;
        nins += N.template insert<EXACTK>(sq_dist(qx, qy, qz, c), r, k);
      }
    }
  }

  if (COUNT) {
    a.cnt_entries[qi] = nent;
    a.cnt_lists[qi] = nlist;
    if (a.cnt_inserts) a.cnt_inserts[qi] = nins;
    return;
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < k) {
      const bool empty = N.r[j] == kEmpty;
      a.out_idx[row + j] = empty ? -1 : N.r[j];
      a.out_dist[row + j] = empty ? INFINITY : (float)sqrt(N.d[j]);
    }
  }
}

// ---------------------------------------------------------------------------------------
// query batch preparation: bucket the queries by the top bits of a 30-bit Morton code of
// their position in the cloud's bounding box (counting sort: histogram, scan, scatter).
// Only locality matters here -- each query's answer does not depend on where it runs.
// ---------------------------------------------------------------------------------------
constexpr int kMortonBits = 18;
constexpr int kMortonBins = 1 << kMortonBits;
// the histogram is scanned in blocks of kScanBlock bins, then over the blocks' totals
constexpr int kScanBlock = 1024;
constexpr int kScanBlocks = kMortonBins / kScanBlock;
static_assert(kScanBlocks <= 1024, "one workgroup scans the block totals");
constexpr int64_t kSortMinQueries = 8192;

// The histogram's atomic hands every query its rank within its bin, so the scatter below
// places it with no atomic of its own.
__global__ __launch_bounds__(256) void morton_hist_kernel(const float *q, int64_t nq, BoxArgs b,
                                                          uint32_t *hist, uint32_t *rank) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  rank[i] = atomicAdd(&hist[morton30(q[3 * i], q[3 * i + 1], q[3 * i + 2], b) >> (30 - kMortonBits)], 1u);
}

// The records of the arena split for the layout measurement: the rank of every record, and,
// when x is given, its coordinates into three arrays.
__global__ __launch_bounds__(256) void split_records_kernel(const float4 *ent, int64_t nrec,
                                                            int32_t *rk, float *x, float *y,
                                                            float *z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrec) return;
  const float4 e = ent[i];
  rk[i] = __float_as_int(e.w);
  if (x) {
    x[i] = e.x;
    y[i] = e.y;
    z[i] = e.z;
  }
}

// Exclusive scan of n counters in place by one workgroup of 1024 threads (n <= 1024); the
// total goes to *total when given.
__device__ __forceinline__ void scan_1024(uint32_t *v, int64_t n, uint32_t *total) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const uint32_t x = t < n ? v[t] : 0u;
  part[t] = x;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t u = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  if (t < n) v[t] = part[t] - x;
  if (total && t == 1023) *total = part[t];
}

// exclusive scan of every block of kScanBlock bins in place; each block's total to sums
__global__ __launch_bounds__(1024) void scan_bins_kernel(uint32_t *hist, uint32_t *sums) {
  scan_1024(hist + (int64_t)blockIdx.x * kScanBlock, kScanBlock, sums + blockIdx.x);
}

// exclusive scan of the kScanBlocks block totals (one workgroup)
__global__ __launch_bounds__(1024) void scan_sums_kernel(uint32_t *sums) {
  scan_1024(sums, kScanBlocks, nullptr);
}

// a bin's first position: its offset in its scan block (start) plus the block's (sums)
__global__ __launch_bounds__(256) void morton_scatter_kernel(const float *q, int64_t nq, BoxArgs b,
                                                             const uint32_t *start,
                                                             const uint32_t *sums,
                                                             const uint32_t *rank, float4 *qs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  float x = q[3 * i], y = q[3 * i + 1], z = q[3 * i + 2];
  const uint32_t bin = morton30(x, y, z, b) >> (30 - kMortonBits);
  const uint32_t pos = start[bin] + sums[bin / kScanBlock] + rank[i];
  qs[pos] = make_float4(x, y, z, __int_as_float((int32_t)i));
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------

static void free_device(mknn_cloud *c) {
  if (c->d_ent) (void)hipFree(c->d_ent);
  if (c->d_lst) (void)hipFree(c->d_lst);
  if (c->d_pts) (void)hipFree(c->d_pts);
  if (c->d_dead) (void)hipFree(c->d_dead);
  if (c->d_overflow) (void)hipFree(c->d_overflow);
  c->d_ent = nullptr;
  c->d_lst = nullptr;
  c->d_pts = nullptr;
  c->d_dead = nullptr;
  c->d_overflow = nullptr;
  c->dead_cap = 0;
  c->dev_bytes = 0;
  c->dev_version = ~0ull;
}

// Deletion deltas: point rank r[t] at its rewritten list segment.
__global__ __launch_bounds__(256) void apply_descriptors_kernel(uint64_t *lst, const int32_t *r,
                                                                const uint64_t *desc, int64_t cnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) lst[r[t]] = desc[t];
}

void release_old_arena(DeviceDelta *d) {
  if (d->old_ent) (void)hipFree(d->old_ent);
  if (d->old_lst) (void)hipFree(d->old_lst);
  if (d->old_pts) (void)hipFree(d->old_pts);
  d->old_ent = nullptr;
  d->old_lst = nullptr;
  d->old_pts = nullptr;
}

// ---- the device image of the lists
mknn_status pack_lists(mknn_cloud *c, HostPack *p) {
  try {
    const int64_t n = c->n;
    // list placement: owners in Morton order
    BoxArgs b = box_of(c);
    std::vector<uint64_t> key(n);
    for (int64_t r = 0; r < n; ++r) {
      const uint64_t code = morton30(c->xyz[3 * r], c->xyz[3 * r + 1], c->xyz[3 * r + 2], b);
      key[r] = (code << 32) | (uint64_t)r;
    }
    std::sort(key.begin(), key.end());
    refresh_csr(c);
    const int64_t nnz = (int64_t)c->succ.ent.size();
    // slack for list rewrites after deletions (copy-on-write segments): half the records.
    // A deleted point rewrites about 25 lists of about 7.5 entries, so this covers deleting
    // about 2% of the points before a re-pack.
    const int64_t cap = nnz + std::max<int64_t>(nnz / 2, 1 << 16) + kEntPad;
    if (cap > (int64_t)0xffffffffll)
      return set_error(MKNN_EUNSUPPORTED, "mknn_upload: more than 2^32 list entries");
    p->ent.assign((size_t)(nnz + kEntPad) * 4, 0.f);
    p->lst.resize((size_t)n);
    p->pts.assign((size_t)n * 4, 0.f);
    for (int64_t r = 0; r < n; ++r)
      for (int k = 0; k < 3; ++k) p->pts[4 * r + k] = c->xyz[3 * r + k];
    uint64_t cur = 0;
    for (int64_t t = 0; t < n; ++t) {
      int64_t r = (int64_t)(key[t] & 0xffffffffu);
      int64_t b0 = c->succ.off[r], b1 = c->succ.off[r + 1];
      p->lst[r] = cur | ((uint64_t)(b1 - b0) << 32);
      for (int64_t e = b0; e < b1; ++e) {
        int32_t j = c->succ.ent[e];
        float *v = &p->ent[cur * 4];
        v[0] = c->xyz[3 * (int64_t)j];
        v[1] = c->xyz[3 * (int64_t)j + 1];
        v[2] = c->xyz[3 * (int64_t)j + 2];
        std::memcpy(&v[3], &j, 4);
        ++cur;
      }
    }
    for (int q = 0; q < kEntPad; ++q) {
      const int32_t big = kEmpty;
      std::memcpy(&p->ent[(cur + q) * 4 + 3], &big, 4);
    }
    p->nnz = nnz;
    p->cap = cap;
  } catch (const std::bad_alloc &) {
    return set_error(MKNN_ENOMEM, "mknn_upload: out of host memory");
  }
  return MKNN_OK;
}

// Allocate a new arena for `p` on the current device and enqueue its copy on `s`.  The
// host image must stay alive until `s` has passed the copies.  The previous arena is not
// touched; c->d_ent / c->d_lst are replaced.
mknn_status install_pack(mknn_cloud *c, const HostPack *p, hipStream_t s) {
  void *ent = nullptr, *pts = nullptr;
  uint64_t *lst = nullptr;
  // descriptors and points for appended ranks: an eighth more than the points present
  const int64_t lst_cap = (int64_t)p->lst.size() + std::max<int64_t>((int64_t)p->lst.size() / 8, 1024);
  hipError_t e = hipMalloc(&ent, sizeof(float4) * (size_t)p->cap);
  if (e == hipSuccess) e = hipMalloc((void **)&lst, sizeof(uint64_t) * (size_t)lst_cap);
  if (e == hipSuccess) e = hipMalloc(&pts, sizeof(float4) * (size_t)lst_cap);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ent, p->ent.data(), sizeof(float) * p->ent.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(lst, p->lst.data(), sizeof(uint64_t) * p->lst.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(pts, p->pts.data(), sizeof(float) * p->pts.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    if (ent) (void)hipFree(ent);
    if (lst) (void)hipFree(lst);
    if (pts) (void)hipFree(pts);
    return set_error(e == hipErrorOutOfMemory ? MKNN_ENOMEM : MKNN_EHIP,
                     std::string("mknn_upload: ") + hipGetErrorName(e));
  }
  c->d_ent = ent;
  c->d_lst = lst;
  c->d_pts = pts;
  c->dev_bytes = (int64_t)(sizeof(float4) * (size_t)p->cap +
                           (sizeof(uint64_t) + sizeof(float4)) * (size_t)lst_cap);
  c->lst_cap = lst_cap;
  c->ent_used = p->nnz;
  c->ent_cap = p->cap - kEntPad;
  note_device_state(c);
  c->dev_version = c->version.load();
  return MKNN_OK;
}

// ---- deletion: host preparation and device application of the list deltas
// The device side of a list change on the host (deletion or insertion): `changed` lists
// are copied on write into fresh arena segments, or -- when the arena's slack or the
// descriptor array would run out -- a complete new image is built here, off the caller's
// launch path.
static mknn_status fill_delta(mknn_cloud *c, const std::vector<int32_t> &changed, DeviceDelta *d,
                              const char *who) {
  int64_t need = 0;
  for (int32_t r : changed) need += c->dsucc.size(r);
  if (c->ent_used + need > c->ent_cap || c->n > c->lst_cap) {
    d->repack = true;
    mknn_status st = pack_lists(c, &d->pack);
    if (st != MKNN_OK) ++c->version;   // the host lists have moved on without the device
    return st;
  }
  try {
    // appended points (insertion), for the per-rank point array
    d->pts_from = c->dev_n;
    d->new_pts.assign((size_t)(c->n - c->dev_n) * 4, 0.f);
    for (int64_t r = c->dev_n; r < c->n; ++r)
      for (int k = 0; k < 3; ++k) d->new_pts[4 * (r - c->dev_n) + k] = c->xyz[3 * r + k];
    // copy-on-write: every changed list gets a fresh segment at the end of the arena, so
    // work that already read the old descriptor keeps reading the old, untouched records
    d->ranks = changed;
    d->lens.resize(changed.size());
    d->rec.resize((size_t)need * 4);
    int64_t cur = 0;
    for (size_t t = 0; t < changed.size(); ++t) {
      const int32_t r = changed[t];
      const int32_t len = c->dsucc.size(r);
      const int32_t *b = c->dsucc.begin(r);
      d->lens[t] = (uint32_t)len;
      for (int32_t e = 0; e < len; ++e) {
        const int32_t j = b[e];
        float *v = &d->rec[(size_t)(cur + e) * 4];
        v[0] = c->xyz[3 * (int64_t)j];
        v[1] = c->xyz[3 * (int64_t)j + 1];
        v[2] = c->xyz[3 * (int64_t)j + 2];
        std::memcpy(&v[3], &j, 4);
      }
      cur += len;
    }
  } catch (const std::bad_alloc &) {
    ++c->version;
    return set_error(MKNN_ENOMEM, std::string(who) + ": out of host memory");
  }
  return MKNN_OK;
}

mknn_status delete_prepare(mknn_cloud *c, const int32_t *ranks, int64_t count, DeviceDelta *d) {
  d->on_device = c->d_ent && c->dev_version == c->version;
  std::vector<int32_t> changed;
  mknn_status st = delete_ranks_host(c, ranks, count, &changed);
  if (st != MKNN_OK) return st;   // a half-applied batch has bumped c->version
  if (!d->on_device) {
    ++c->version;
    return MKNN_OK;
  }
  // on the device the version moves when the delta is applied
  return fill_delta(c, changed, d, "mknn_delete");
}

mknn_status insert_prepare(mknn_cloud *c, const float *xyz, int64_t count, DeviceDelta *d) {
  d->on_device = c->d_ent && c->dev_version == c->version;
  std::vector<int32_t> changed;
  mknn_status st = insert_points_host(c, xyz, count, &changed);
  if (st != MKNN_OK) return st;   // a half-applied batch has bumped c->version
  if (!d->on_device) {
    ++c->version;
    return MKNN_OK;
  }
  return fill_delta(c, changed, d, "mknn_insert");
}

mknn_status apply_delta(mknn_cloud *c, DeviceDelta *d, hipStream_t s) {
  if (!d->on_device) return MKNN_OK;
  ++c->version;   // the device copy is stale until the delta below is complete
  const int64_t need = (int64_t)(d->rec.size() / 4);
  if (d->repack) {
    // a new arena; the old one is kept for the work that still reads it (d->old_*)
    void *old_ent = c->d_ent, *old_pts = c->d_pts;
    uint64_t *old_lst = c->d_lst;
    mknn_status st = install_pack(c, &d->pack, s);
    if (st != MKNN_OK) return st;
    d->old_ent = old_ent;
    d->old_lst = old_lst;
    d->old_pts = old_pts;
    return MKNN_OK;
  }
  if (d->ranks.empty() && need == 0 && d->new_pts.empty()) {
    // nothing changed (an empty batch)
    note_device_state(c);
    c->dev_version = c->version.load();
    return MKNN_OK;
  }
  d->desc.resize(d->ranks.size());
  int64_t cur = 0;
  for (size_t t = 0; t < d->ranks.size(); ++t) {
    d->desc[t] = (uint64_t)(c->ent_used + cur) | ((uint64_t)d->lens[t] << 32);
    cur += d->lens[t];
  }
  void *d_tmp = nullptr;
  const size_t tmp_bytes = sizeof(int32_t) * d->ranks.size() + sizeof(uint64_t) * d->desc.size() + 16;
  HIP_TRY(hipMallocAsync(&d_tmp, tmp_bytes, s), "apply list delta: scratch");
  uint64_t *d_dd = (uint64_t *)d_tmp;
  int32_t *d_rr = (int32_t *)(d_dd + d->desc.size());
  if (need)
    HIP_TRY(hipMemcpyAsync((float4 *)c->d_ent + c->ent_used, d->rec.data(), sizeof(float) * d->rec.size(),
                           hipMemcpyHostToDevice, s), "apply list delta: copy records");
  if (!d->new_pts.empty())
    HIP_TRY(hipMemcpyAsync((float4 *)c->d_pts + d->pts_from, d->new_pts.data(),
                           sizeof(float) * d->new_pts.size(), hipMemcpyHostToDevice, s),
            "apply list delta: copy points");
  HIP_TRY(hipMemcpyAsync(d_dd, d->desc.data(), sizeof(uint64_t) * d->desc.size(), hipMemcpyHostToDevice, s),
          "apply list delta: copy descriptors");
  HIP_TRY(hipMemcpyAsync(d_rr, d->ranks.data(), sizeof(int32_t) * d->ranks.size(), hipMemcpyHostToDevice, s),
          "apply list delta: copy ranks");
  const uint32_t blocks = (uint32_t)((d->ranks.size() + 255) / 256);
  hipLaunchKernelGGL(apply_descriptors_kernel, dim3(blocks), dim3(256), 0, s, c->d_lst, d_rr, d_dd,
                     (int64_t)d->ranks.size());
  HIP_TRY(hipGetLastError(), "apply list delta: launch");
  HIP_TRY(hipFreeAsync(d_tmp, s), "apply list delta: free scratch");
  c->ent_used += need;
  note_device_state(c);
  c->dev_version = c->version.load();
  return MKNN_OK;
}

// ---- optional kernel timing
static bool g_timing = false;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;
static size_t g_events_used = 0;

bool timing_enabled() { return g_timing; }

hipError_t timing_mark(hipStream_t s, bool start) {
  if (!g_timing) return hipSuccess;
  if (start) {
    if (g_events_used == g_events.size()) {
      hipEvent_t a, b;
      hipError_t e = hipEventCreate(&a);
      if (e != hipSuccess) return e;
      e = hipEventCreate(&b);
      if (e != hipSuccess) return e;
      g_events.push_back({a, b});
    }
    return hipEventRecord(g_events[g_events_used].first, s);
  }
  return hipEventRecord(g_events[g_events_used++].second, s);
}

// ---------------------------------------------------------------------------------------
// Launch configuration and the autotuner's table
//
// A configuration picks the kernel family (1: one query per lane, 2: 16 lanes per query in
// lockstep, 3: 16 lanes per query with independently scheduled rows), the number of
// candidates per chunk from which k <= 16 merges with the network instead of inserting one
// by one, and the queries per wavefront of the row kernel.  mknn_autotune fills a table
// keyed by (device, slots per lane S, k == 16 S, log2 n); launches look their key up and
// fall back to the measured defaults.  Environment variables override both (experiments).
// ---------------------------------------------------------------------------------------
static long env_long(const char *name, long dflt) {
  const char *e = getenv(name);
  return e ? atol(e) : dflt;
}

// Defaults measured on the 1M torus: scheduled rows, one query per row, and the merge
// network from 6 / 8 / 8 / 8 candidates per chunk for S = 1..4 slots per lane.
static TuneConfig default_config(int S) {
  static const int32_t mm[4] = {8, 8, 8, 8};
  return {3, mm[(S < 1 ? 1 : S > 4 ? 4 : S) - 1], 4};
}

static std::mutex g_tune_mu;
static std::map<uint64_t, TuneConfig> g_tune;

static uint64_t tune_key(int dev, int S, bool exact, int64_t n) {
  int b = 0;
  while (b < 40 && ((int64_t)1 << (b + 1)) <= n) ++b;
  return ((uint64_t)(uint32_t)dev << 32) | ((uint64_t)S << 16) | ((uint64_t)(exact ? 1 : 0) << 8) |
         (uint64_t)b;
}

static TuneConfig env_overrides(TuneConfig c) {
  static long fam = -2, mm = -2, pw = -2;
  if (fam == -2) {
    const char *v = getenv("MKNN_KERNEL");
    fam = (v && v[0] == 'l') ? 1 : (v && v[0] == 'g') ? 2 : (v && v[0] == 'r') ? 3 : 0;
    mm = env_long("MKNN_MERGE_MIN", 0);
    pw = env_long("MKNN_PER_WAVE", 0);
  }
  if (fam > 0) c.family = (int32_t)fam;
  if (mm > 0) c.merge_min = (int32_t)mm;
  if (pw >= 4) c.per_wave = (int32_t)pw;
  return c;
}

TuneConfig config_for(int kmax, bool exact, int64_t n) {
  const int S = (kmax + 15) / 16;
  int dev = 0;
  (void)hipGetDevice(&dev);
  TuneConfig c = default_config(S);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(dev, S, exact && kmax == 16 * S, n));
    if (it != g_tune.end()) c = it->second;
  }
  return env_overrides(c);
}

template <int K, bool EXACTK, bool COUNT>
static hipError_t launch_lane(const QueryArgs &a, hipStream_t s) {
  const int threads = 256;
  const uint32_t blocks = (uint32_t)((a.nq + threads - 1) / threads);
  hipLaunchKernelGGL((knn_lane_kernel<K, EXACTK, COUNT>), dim3(blocks), dim3(threads), 0, s, a);
  return hipGetLastError();
}

template <bool COUNT>
static hipError_t dispatch_lane(const QueryArgs &a, int kmax, bool exact, hipStream_t s) {
#define MKNN_CASE(KK)                                                                       \
  if (kmax <= KK)                                                                          \
    return (exact && kmax == KK) ? launch_lane<KK, true, COUNT>(a, s)                     \
                                 : launch_lane<KK, false, COUNT>(a, s);
  MKNN_CASE(1)
  MKNN_CASE(2)
  MKNN_CASE(4)
  MKNN_CASE(8)
  MKNN_CASE(16)
  MKNN_CASE(32)
  MKNN_CASE(64)
#undef MKNN_CASE
  return hipErrorInvalidValue;
}

// Optional dynamic LDS per workgroup of the group kernel, used only to cap occupancy in
// experiments (MKNN_LDS_PAD bytes).
static size_t lds_pad() {
  static long v = -1;
  if (v < 0) v = env_long("MKNN_LDS_PAD", 0);
  return (size_t)v;
}

template <int S, bool EXACTK, bool COUNT>
static hipError_t launch_group(const QueryArgs &a, hipStream_t s) {
  const int threads = 256;   // 4 waves x 4 queries
  const uint32_t blocks = (uint32_t)((a.nq + 15) / 16);
  hipLaunchKernelGGL((knn_group_kernel<S, EXACTK, COUNT>), dim3(blocks), dim3(threads), lds_pad(),
                     s, a);
  return hipGetLastError();
}

template <bool COUNT>
static hipError_t dispatch_group(const QueryArgs &a, int kmax, bool exact, hipStream_t s) {
#define MKNN_GCASE(SS)                                                                      \
  if (kmax <= 16 * SS)                                                                     \
    return (exact && kmax == 16 * SS) ? launch_group<SS, true, COUNT>(a, s)               \
                                      : launch_group<SS, false, COUNT>(a, s);
  MKNN_GCASE(1)
  MKNN_GCASE(2)
  MKNN_GCASE(3)
  MKNN_GCASE(4)
#undef MKNN_GCASE
  return hipErrorInvalidValue;
}

template <int S, bool EXACTK>
static hipError_t launch_rows(const QueryArgs &a, int32_t per_wave, hipStream_t s) {
  const int64_t waves = (a.nq + per_wave - 1) / per_wave;
  const uint32_t blocks = (uint32_t)((waves + 3) / 4);
  // descent steps first only when every row keeps its one query for the whole launch;
  // k and m as scalars when there are no per-query arrays (always so for exact k)
  const bool uniform = !a.kq && !a.mq;
  if (a.dead) {
    // pending deletions: the filtering variants (descent first, one query per row)
    if (per_wave != 4) return hipErrorInvalidValue;
    if (EXACTK || uniform)
      hipLaunchKernelGGL((knn_rows_kernel<S, EXACTK, true, true, true>), dim3(blocks), dim3(256), 0, s, a, per_wave);
    else if constexpr (!EXACTK)
      hipLaunchKernelGGL((knn_rows_kernel<S, false, true, false, true>), dim3(blocks), dim3(256), 0, s, a, per_wave);
  } else if (EXACTK || uniform) {
    if (per_wave == 4)
      hipLaunchKernelGGL((knn_rows_kernel<S, EXACTK, true, true>), dim3(blocks), dim3(256), 0, s, a, per_wave);
    else
      hipLaunchKernelGGL((knn_rows_kernel<S, EXACTK, false, true>), dim3(blocks), dim3(256), 0, s, a, per_wave);
  } else if constexpr (!EXACTK) {
    if (per_wave == 4)
      hipLaunchKernelGGL((knn_rows_kernel<S, false, true, false>), dim3(blocks), dim3(256), 0, s, a, per_wave);
    else
      hipLaunchKernelGGL((knn_rows_kernel<S, false, false, false>), dim3(blocks), dim3(256), 0, s, a, per_wave);
  }
  return hipGetLastError();
}

static hipError_t dispatch_rows(const QueryArgs &a, int kmax, bool exact, int32_t per_wave,
                                hipStream_t s) {
#define MKNN_RCASE(SS)                                                                      \
  if (kmax <= 16 * SS)                                                                     \
    return (exact && kmax == 16 * SS) ? launch_rows<SS, true>(a, per_wave, s)             \
                                      : launch_rows<SS, false>(a, per_wave, s);
  MKNN_RCASE(1)
  MKNN_RCASE(2)
  MKNN_RCASE(3)
  MKNN_RCASE(4)
#undef MKNN_RCASE
  return hipErrorInvalidValue;
}

// Bytes of scratch the Morton bucketing of nq queries needs (0 below the sort threshold).
static size_t sort_scratch_bytes(int64_t nq) {
  return nq < kSortMinQueries ? 0
                              : sizeof(uint32_t) * (kMortonBins + kScanBlocks) +
                                    (sizeof(float4) + sizeof(uint32_t)) * (size_t)nq;
}

// Morton bucketing of the queries, for batches large enough to pay for it.  The scratch
// (sort_scratch_bytes(nq), 256-byte aligned) comes from `fixed` when given, else from the
// stream-ordered allocator (returned in *scratch for the caller to release).
static mknn_status prepare_queries(const mknn_cloud *c, const float *d_q, int64_t nq,
                                   hipStream_t s, float4 **qs_out, void **scratch,
                                   void *fixed = nullptr) {
  *qs_out = nullptr;
  *scratch = nullptr;
  if (nq < kSortMinQueries) return MKNN_OK;
  uint32_t *hist = (uint32_t *)fixed;
  if (!hist) {
    HIP_TRY(hipMallocAsync(scratch, sort_scratch_bytes(nq), s), "query sort scratch");
    hist = (uint32_t *)*scratch;
  }
  uint32_t *sums = hist + kMortonBins;
  float4 *qs = (float4 *)(sums + kScanBlocks);
  uint32_t *rank = (uint32_t *)(qs + nq);
  BoxArgs b = dev_box_of(c);
  const int threads = 256;
  const uint32_t blocks = (uint32_t)((nq + threads - 1) / threads);
  hipLaunchKernelGGL(fill_kernel<uint32_t>, dim3(kMortonBins / threads), dim3(threads), 0, s,
                     hist, (int64_t)kMortonBins, 0u);
  hipLaunchKernelGGL(morton_hist_kernel, dim3(blocks), dim3(threads), 0, s, d_q, nq, b, hist, rank);
  hipLaunchKernelGGL(scan_bins_kernel, dim3(kScanBlocks), dim3(1024), 0, s, hist, sums);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, sums);
  hipLaunchKernelGGL(morton_scatter_kernel, dim3(blocks), dim3(threads), 0, s, d_q, nq, b, hist,
                     sums, rank, qs);
  HIP_TRY(hipGetLastError(), "query sort launch");
  *qs_out = qs;
  return MKNN_OK;
}

// Pending deletions on a launch: the walk collects kout + kLazyMargin neighbours (at most
// MKNN_KMAX) and the rows keep the first kout unmarked ones (QueryArgs::dead).
struct LazyLaunch {
  int32_t kout;
  uint32_t epoch;   // filter the marks of epochs 1 .. epoch
};

static mknn_status run_query(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k,
                             int32_t m, const int32_t *d_k, const int32_t *d_m,
                             const int64_t *d_row_off, int32_t kmax, int32_t *d_idx,
                             float *d_dist, int32_t *d_ce, int32_t *d_cl, int32_t *d_ci,
                             hipStream_t s, const char *who, const TuneConfig *force = nullptr,
                             float *d_plane = nullptr, void *fixed_scratch = nullptr,
                             const LazyLaunch *lazy = nullptr) {
  QueryArgs a;
  fill_cloud_args(c, &a);
  if (lazy) {
    a.dead = c->d_dead;
    a.kout = lazy->kout;
    a.epoch = lazy->epoch;
    a.overflow = c->d_overflow;
  }
  a.q = d_q;
  a.nq = nq;
  a.k = k;
  a.m = m;
  a.kq = d_k;
  a.mq = d_m;
  a.row_off = d_row_off;
  a.out_idx = d_idx;
  a.out_dist = d_dist;
  a.cnt_entries = d_ce;
  a.cnt_lists = d_cl;
  a.cnt_inserts = d_ci;
  void *scratch = nullptr;
  float4 *qs = nullptr;
  mknn_status st = prepare_queries(c, d_q, nq, s, &qs, &scratch, fixed_scratch);
  if (st != MKNN_OK) return st;
  a.qs = qs;
  const bool exact = (d_k == nullptr);
  TuneConfig cfg = force ? *force : config_for(kmax, exact, c->dev_n);
  if (lazy) {
    cfg.family = 3;   // only the row kernels filter marked ranks
    cfg.per_wave = 4;
  }
  a.merge_min = cfg.merge_min;
  // the allocation-free entry point records no timing events (they are created on demand)
  hipError_t e = fixed_scratch ? hipSuccess : timing_mark(s, true);
  if (e == hipSuccess) {
    if (cfg.family == 1)
      e = d_ce ? dispatch_lane<true>(a, kmax, exact, s) : dispatch_lane<false>(a, kmax, exact, s);
    else if (cfg.family == 3 && !d_ce)
      e = dispatch_rows(a, kmax, exact, cfg.per_wave, s);
    else
      e = d_ce ? dispatch_group<true>(a, kmax, exact, s) : dispatch_group<false>(a, kmax, exact, s);
  }
  if (e == hipSuccess && !fixed_scratch) e = timing_mark(s, false);
  // the plane fit reads the rows just written (and the sorted queries, for their order)
  if (e == hipSuccess && d_plane)
    e = launch_plane_fit((const float4 *)c->d_pts, d_idx, qs, nq, lazy ? lazy->kout : k, d_plane, s);
  if (scratch) (void)hipFreeAsync(scratch, s);
  if (e != hipSuccess)
    return set_error(MKNN_EHIP, std::string(who) + ": launch failed: " + hipGetErrorName(e));
  return MKNN_OK;
}

// Per-query arguments of mknn_knn_var: the smallest index of a query whose k lies outside
// [1, kmax], whose m is below 1, or whose row length differs from its k.
__global__ __launch_bounds__(256) void check_per_query_kernel(const int32_t *kq, const int32_t *mq,
                                                              const int64_t *off, int64_t nq,
                                                              int32_t kmax, int32_t *first_bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int32_t k = kq[i], m = mq[i];
  const int64_t a = off[i], b = off[i + 1];
  if (k < 1 || k > kmax || m < 1 || a < 0 || b - a != (int64_t)k) atomicMin(first_bad, (int32_t)i);
}

// Checks the per-query arrays on the device and reads the verdict back (synchronises s).
static mknn_status check_per_query(const int32_t *d_k, const int32_t *d_m, const int64_t *d_off,
                                   int64_t nq, int32_t kmax, hipStream_t s) {
  int32_t *flag = nullptr;
  HIP_TRY(hipMallocAsync((void **)&flag, sizeof(int32_t), s), "mknn_knn_var: check scratch");
  hipLaunchKernelGGL(fill_kernel<int32_t>, dim3(1), dim3(64), 0, s, flag, (int64_t)1,
                     (int32_t)0x7fffffff);
  hipLaunchKernelGGL(check_per_query_kernel, dim3((uint32_t)((nq + 255) / 256)), dim3(256), 0, s,
                     d_k, d_m, d_off, nq, kmax, flag);
  int32_t bad = 0x7fffffff;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  (void)hipFreeAsync(flag, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess)
    return set_error(MKNN_EHIP, std::string("mknn_knn_var: argument check: ") + hipGetErrorName(e));
  if (bad != 0x7fffffff) {
    int32_t k = 0, m = 0;
    int64_t off[2] = {0, 0};
    (void)hipMemcpy(&k, d_k + bad, sizeof(k), hipMemcpyDeviceToHost);
    (void)hipMemcpy(&m, d_m + bad, sizeof(m), hipMemcpyDeviceToHost);
    (void)hipMemcpy(off, d_off + bad, sizeof(off), hipMemcpyDeviceToHost);
    return set_error(MKNN_EINVAL, "mknn_knn_var: query " + std::to_string(bad) + " has k=" +
                                      std::to_string(k) + " (kmax " + std::to_string(kmax) +
                                      "), m=" + std::to_string(m) + ", row length " +
                                      std::to_string(off[1] - off[0]));
  }
  return MKNN_OK;
}

// ---------------------------------------------------------------------------------------
// Allocation-free variant of mknn_knn: the query sort's scratch is a fixed device array of
// this translation unit (one copy per GPU, held until the process ends) instead of
// stream-ordered allocations.  Host code never passes the array's name to a kernel: the
// name is a host-side stand-in, and its device address comes from hipGetSymbolAddress, once
// per device with that device current.
// ---------------------------------------------------------------------------------------
constexpr int64_t kStaticMaxQueries = (int64_t)1 << 20;
constexpr size_t kStaticScratchBytes = sizeof(uint32_t) * (kMortonBins + kScanBlocks) +
                                       (sizeof(float4) + sizeof(uint32_t)) * (size_t)kStaticMaxQueries;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (looked up on the first call there).
static mknn_status static_scratch(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "mknn_knn_static: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(MKNN_EUNSUPPORTED, "mknn_knn_static: device ordinal above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "mknn_knn_static: hipGetSymbolAddress");
    if (!p) return set_error(MKNN_EHIP, "mknn_knn_static: scratch has no device address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MKNN_OK;
}

// ---------------------------------------------------------------------------------------
// Pending (lazy) deletions
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mark_dead_kernel(uint32_t *dead, const int32_t *r,
                                                        int64_t cnt, uint32_t epoch) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) dead[r[i]] = epoch;
}

mknn_status ensure_epochs_async(mknn_cloud *c, int64_t need, hipStream_t s, uint32_t **old) {
  *old = nullptr;
  if (c->d_dead && c->dead_cap >= need) return MKNN_OK;
  const int64_t cap = std::max<int64_t>(2 * need, 4096);
  uint32_t *nd = nullptr;
  HIP_TRY(hipMalloc((void **)&nd, sizeof(uint32_t) * (size_t)cap), "deletion epochs");
  hipLaunchKernelGGL(fill_kernel<uint32_t>, dim3(256), dim3(256), 0, s, nd, cap, 0u);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && c->d_dead)
    e = hipMemcpyAsync(nd, c->d_dead, sizeof(uint32_t) * (size_t)c->dead_cap,
                       hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(nd);
    return set_error(MKNN_EHIP, std::string("deletion epochs: ") + hipGetErrorName(e));
  }
  *old = c->d_dead;
  c->d_dead = nd;
  c->dead_cap = cap;
  return MKNN_OK;
}

mknn_status mark_deleted_async(mknn_cloud *c, const int32_t *ranks, int64_t count,
                               uint32_t epoch, hipStream_t s) {
  if (count == 0) return MKNN_OK;
  int32_t *d_r = nullptr;
  HIP_TRY(hipMallocAsync((void **)&d_r, sizeof(int32_t) * (size_t)count, s), "mark deletions");
  hipError_t e = hipMemcpyAsync(d_r, ranks, sizeof(int32_t) * (size_t)count, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(mark_dead_kernel, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, s,
                       c->d_dead, d_r, count, epoch);
    e = hipGetLastError();
  }
  (void)hipFreeAsync(d_r, s);
  if (e != hipSuccess) return set_error(MKNN_EHIP, std::string("mark deletions: ") + hipGetErrorName(e));
  return MKNN_OK;
}

// Applies the pending deletions (Alg. 3 on the host, the delta on s); synchronises s.
mknn_status flush_pending(mknn_cloud *c, hipStream_t s, const int32_t *more, int64_t nmore) {
  std::vector<int32_t> all(c->lazy);
  if (more) all.insert(all.end(), more, more + nmore);
  if (all.empty()) return MKNN_OK;
  DeviceDelta d;
  const uint64_t version = c->version;
  mknn_status st = delete_prepare(c, all.data(), (int64_t)all.size(), &d);
  // a batch that changed nothing keeps the pending set; one applied (even in part) ends it
  if (st != MKNN_OK && c->version == version) return st;
  for (int32_t r : c->lazy) c->lazy_mark[r] = 0;
  c->lazy.clear();
  c->dev_lazy = 0;
  if (st != MKNN_OK) return st;
  if (!d.on_device) return MKNN_OK;
  st = apply_delta(c, &d, s);
  if (st != MKNN_OK) return st;
  HIP_TRY(hipStreamSynchronize(s), "apply pending deletions: synchronize");
  release_old_arena(&d);
  return MKNN_OK;
}

// A query call on the device lists.  With pending deletions the launch over-fetches and
// filters (LazyLaunch), then the overflow counter is read back (s is synchronised) and, if
// some row could not be certified, the pending deletions are applied and the call runs
// again on the new lists.  launch(const LazyLaunch *) enqueues the call.
template <typename Launch>
static mknn_status run_with_pending(const mknn_cloud *cc, int32_t kout, hipStream_t s,
                                    const char *who, Launch launch) {
  mknn_cloud *c = const_cast<mknn_cloud *>(cc);
  if (c->dev_lazy.load() == 0 || !c->d_dead) return launch(nullptr);
  const LazyLaunch lz{kout, c->lazy_epoch};
  hipLaunchKernelGGL(fill_kernel<uint32_t>, dim3(1), dim3(64), 0, s, c->d_overflow, (int64_t)1, 0u);
  mknn_status st = launch(&lz);
  if (st != MKNN_OK) return st;
  uint32_t ovf = 0;
  HIP_TRY(hipMemcpyAsync(&ovf, c->d_overflow, sizeof(ovf), hipMemcpyDeviceToHost, s), who);
  HIP_TRY(hipStreamSynchronize(s), who);
  if (ovf == 0) return MKNN_OK;
  st = flush_pending(c, s);
  if (st != MKNN_OK) return st;
  return launch(nullptr);
}

}  // namespace mknn

using namespace mknn;

extern "C" {

mknn_status mknn_upload(mknn_cloud *c, void *stream) {
  clear_error();
  if (!c) return set_error(MKNN_EINVAL, "mknn_upload: cloud is NULL");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "mknn_upload: hipGetDevice");
  if (c->d_ent && c->dev_version == c->version && c->device == dev) return MKNN_OK;
  hipStream_t s = (hipStream_t)stream;
  mknn_status st = MKNN_OK;
  if (!c->lazy.empty()) {
    // pending deletions are applied to the host lists only; the new copy then holds them
    free_device(c);
    st = flush_pending(c, s);
    if (st != MKNN_OK) return st;
  }
  HostPack pack;
  st = pack_lists(c, &pack);
  if (st != MKNN_OK) return st;
  free_device(c);
  c->device = dev;
  st = install_pack(c, &pack, s);
  if (st != MKNN_OK) return st;
  HIP_TRY(hipStreamSynchronize(s), "mknn_upload: synchronize");
  return MKNN_OK;
}

mknn_status mknn_compact(mknn_cloud *c, void *stream) {
  clear_error();
  if (!c) return set_error(MKNN_EINVAL, "mknn_compact: cloud is NULL");
  mknn_status st = check_uploaded(c, "mknn_compact");
  if (st != MKNN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  HostPack pack;
  st = pack_lists(c, &pack);
  if (st != MKNN_OK) return st;
  DeviceDelta old;
  old.old_ent = c->d_ent;
  old.old_lst = c->d_lst;
  old.old_pts = c->d_pts;
  st = install_pack(c, &pack, s);
  if (st != MKNN_OK) return st;
  HIP_TRY(hipStreamSynchronize(s), "mknn_compact: synchronize");
  release_old_arena(&old);
  return MKNN_OK;
}

int64_t mknn_device_bytes(const mknn_cloud *c) { return c ? c->dev_bytes : 0; }

mknn_status mknn_knn(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k, int32_t m,
                     int32_t *d_idx, float *d_dist, void *stream) {
  clear_error();
  if (k > MKNN_KMAX) return set_error(MKNN_EUNSUPPORTED, "mknn_knn: k above MKNN_KMAX");
  if (k < 1) return set_error(MKNN_EINVAL, "mknn_knn: k must be >= 1");
  if (nq < 0 || nq > 0x7fffffffll) return set_error(MKNN_EINVAL, "mknn_knn: nq out of range");
  mknn_status st = check_uploaded(c, "mknn_knn");
  if (st != MKNN_OK) return st;
  if (m < 1 || m > c->dev_n) return set_error(MKNN_EINVAL, "mknn_knn: m must be in [1, n]");
  if (nq == 0) return MKNN_OK;
  if (!d_q || !d_idx || !d_dist) return set_error(MKNN_EINVAL, "mknn_knn: NULL buffer");
  hipStream_t s = (hipStream_t)stream;
  return run_with_pending(c, k, s, "mknn_knn", [&](const LazyLaunch *lz) {
    const int32_t kw = lz ? std::min<int32_t>(MKNN_KMAX, k + kLazyMargin) : k;
    return run_query(c, d_q, nq, kw, m, nullptr, nullptr, nullptr, kw, d_idx, d_dist, nullptr,
                     nullptr, nullptr, s, "mknn_knn", nullptr, nullptr, nullptr, lz);
  });
}

mknn_status mknn_knn_layout(const mknn_cloud *c, int32_t layout, const float *d_q, int64_t nq,
                            int32_t *d_idx, float *d_dist, void *stream) {
  clear_error();
  if (layout != MKNN_LAYOUT_RANKS && layout != MKNN_LAYOUT_ARRAYS)
    return set_error(MKNN_EINVAL, "mknn_knn_layout: layout must be MKNN_LAYOUT_RANKS or "
                                  "MKNN_LAYOUT_ARRAYS");
  if (nq < 0 || nq > 0x7fffffffll)
    return set_error(MKNN_EINVAL, "mknn_knn_layout: nq out of range");
  mknn_status st = check_uploaded(c, "mknn_knn_layout");
  if (st != MKNN_OK) return st;
  if (nq == 0) return MKNN_OK;
  if (!d_q || !d_idx || !d_dist)
    return set_error(MKNN_EINVAL, "mknn_knn_layout: NULL buffer");
  if (c->dev_lazy.load() != 0)
    return set_error(MKNN_EUNSUPPORTED, "mknn_knn_layout: the cloud has pending deletions");
  hipStream_t s = (hipStream_t)stream;
  // the other layout of every record, padding included: 4 bytes of rank, and for the four
  // arrays 12 more bytes of coordinates
  const bool arrays = layout == MKNN_LAYOUT_ARRAYS;
  const int64_t nrec = c->ent_cap + kEntPad;
  const size_t per = arrays ? 16 : 4;
  char *buf = nullptr;
  HIP_TRY(hipMallocAsync((void **)&buf, per * (size_t)nrec, s), "mknn_knn_layout: arrays");
  int32_t *rk = (int32_t *)buf;
  float *sx = arrays ? (float *)(buf + 4 * (size_t)nrec) : nullptr;
  float *sy = arrays ? (float *)(buf + 8 * (size_t)nrec) : nullptr;
  float *sz = arrays ? (float *)(buf + 12 * (size_t)nrec) : nullptr;
  hipLaunchKernelGGL(split_records_kernel, dim3((uint32_t)((nrec + 255) / 256)), dim3(256), 0,
                     s, (const float4 *)c->d_ent, nrec, rk, sx, sy, sz);
  QueryArgs a;
  fill_cloud_args(c, &a);
  a.q = d_q;
  a.nq = nq;
  a.k = 16;
  a.m = (int32_t)c->dev_n;
  a.kq = a.mq = nullptr;
  a.row_off = nullptr;
  a.out_idx = d_idx;
  a.out_dist = d_dist;
  a.cnt_entries = a.cnt_lists = a.cnt_inserts = nullptr;
  a.rk = rk;
  a.pts = (const float4 *)c->d_pts;
  a.sx = sx;
  a.sy = sy;
  a.sz = sz;
  void *scratch = nullptr;
  float4 *qs = nullptr;
  st = prepare_queries(c, d_q, nq, s, &qs, &scratch);
  if (st != MKNN_OK) {
    (void)hipFreeAsync(buf, s);
    return st;
  }
  a.qs = qs;
  a.merge_min = config_for(16, true, c->dev_n).merge_min;
  hipError_t e = timing_mark(s, true);
  const int64_t waves = (nq + 3) / 4;
  const dim3 grid((uint32_t)((waves + 3) / 4));
  if (e == hipSuccess) {
    if (arrays)
      hipLaunchKernelGGL(knn_rows_layout_kernel<kLayoutArrays>, grid, dim3(256), 0, s, a,
                         (int32_t)4);
    else
      hipLaunchKernelGGL(knn_rows_layout_kernel<kLayoutRanks>, grid, dim3(256), 0, s, a,
                         (int32_t)4);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = timing_mark(s, false);
  if (scratch) (void)hipFreeAsync(scratch, s);
  (void)hipFreeAsync(buf, s);
  if (e != hipSuccess)
    return set_error(MKNN_EHIP, std::string("mknn_knn_layout: ") + hipGetErrorName(e));
  return MKNN_OK;
}

mknn_status mknn_knn_static(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k,
                            int32_t m, int32_t *d_idx, float *d_dist, void *stream) {
  clear_error();
  if (k > MKNN_KMAX) return set_error(MKNN_EUNSUPPORTED, "mknn_knn_static: k above MKNN_KMAX");
  if (k < 1) return set_error(MKNN_EINVAL, "mknn_knn_static: k must be >= 1");
  if (nq < 0 || nq > kStaticMaxQueries)
    return set_error(MKNN_EINVAL, "mknn_knn_static: nq must be in [0, " +
                                      std::to_string(kStaticMaxQueries) +
                                      "] (the size of the fixed scratch)");
  mknn_status st = check_uploaded(c, "mknn_knn_static");
  if (st != MKNN_OK) return st;
  if (m < 1 || m > c->dev_n) return set_error(MKNN_EINVAL, "mknn_knn_static: m must be in [1, n]");
  if (nq == 0) return MKNN_OK;
  if (!d_q || !d_idx || !d_dist) return set_error(MKNN_EINVAL, "mknn_knn_static: NULL buffer");
  if (c->dev_lazy.load() != 0)
    return set_error(MKNN_EUNSUPPORTED, "mknn_knn_static: the cloud has pending deletions "
                                        "(apply them with mknn_delete_flush first)");
  void *buf = nullptr;
  st = static_scratch(&buf);
  if (st != MKNN_OK) return st;
  static_assert(kStaticScratchBytes >= sizeof(uint32_t) * (kMortonBins + kScanBlocks) +
                                          (sizeof(float4) + sizeof(uint32_t)) * (size_t)kStaticMaxQueries,
                "scratch holds the sort of the largest batch");
  return run_query(c, d_q, nq, k, m, nullptr, nullptr, nullptr, k, d_idx, d_dist, nullptr,
                   nullptr, nullptr, (hipStream_t)stream, "mknn_knn_static", nullptr, nullptr,
                   buf);
}

mknn_status mknn_knn_plane(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k,
                           int32_t m, int32_t *d_idx, float *d_dist, float *d_plane,
                           void *stream) {
  clear_error();
  if (k > MKNN_KMAX) return set_error(MKNN_EUNSUPPORTED, "mknn_knn_plane: k above MKNN_KMAX");
  if (k < 1) return set_error(MKNN_EINVAL, "mknn_knn_plane: k must be >= 1");
  if (nq < 0 || nq > 0x7fffffffll) return set_error(MKNN_EINVAL, "mknn_knn_plane: nq out of range");
  mknn_status st = check_uploaded(c, "mknn_knn_plane");
  if (st != MKNN_OK) return st;
  if (m < 1 || m > c->dev_n) return set_error(MKNN_EINVAL, "mknn_knn_plane: m must be in [1, n]");
  if (nq == 0) return MKNN_OK;
  if (!d_q || !d_idx || !d_dist || !d_plane)
    return set_error(MKNN_EINVAL, "mknn_knn_plane: NULL buffer");
  hipStream_t s = (hipStream_t)stream;
  return run_with_pending(c, k, s, "mknn_knn_plane", [&](const LazyLaunch *lz) {
    const int32_t kw = lz ? std::min<int32_t>(MKNN_KMAX, k + kLazyMargin) : k;
    return run_query(c, d_q, nq, kw, m, nullptr, nullptr, nullptr, kw, d_idx, d_dist, nullptr,
                     nullptr, nullptr, s, "mknn_knn_plane", nullptr, d_plane, nullptr, lz);
  });
}

mknn_status mknn_knn_var(const mknn_cloud *c, const float *d_q, int64_t nq, const int32_t *d_k,
                         const int32_t *d_m, const int64_t *d_row_off, int32_t kmax,
                         int32_t *d_idx, float *d_dist, void *stream) {
  clear_error();
  if (kmax > MKNN_KMAX) return set_error(MKNN_EUNSUPPORTED, "mknn_knn_var: kmax above MKNN_KMAX");
  if (kmax < 1) return set_error(MKNN_EINVAL, "mknn_knn_var: kmax must be >= 1");
  if (nq < 0 || nq > 0x7fffffffll) return set_error(MKNN_EINVAL, "mknn_knn_var: nq out of range");
  mknn_status st = check_uploaded(c, "mknn_knn_var");
  if (st != MKNN_OK) return st;
  if (nq == 0) return MKNN_OK;
  if (!d_q || !d_k || !d_m || !d_row_off || !d_idx || !d_dist)
    return set_error(MKNN_EINVAL, "mknn_knn_var: NULL buffer");
  hipStream_t s = (hipStream_t)stream;
  st = check_per_query(d_k, d_m, d_row_off, nq, kmax, s);
  if (st != MKNN_OK) return st;
  return run_with_pending(c, 0, s, "mknn_knn_var", [&](const LazyLaunch *lz) {
    const int32_t kw = lz ? std::min<int32_t>(MKNN_KMAX, kmax + kLazyMargin) : kmax;
    return run_query(c, d_q, nq, 0, 0, d_k, d_m, d_row_off, kw, d_idx, d_dist, nullptr, nullptr,
                     nullptr, s, "mknn_knn_var", nullptr, nullptr, nullptr, lz);
  });
}

mknn_status mknn_knn_counts(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k,
                            int32_t m, int32_t *d_entries, int32_t *d_lists, int32_t *d_inserts,
                            void *stream) {
  clear_error();
  if (k > MKNN_KMAX) return set_error(MKNN_EUNSUPPORTED, "mknn_knn_counts: k above MKNN_KMAX");
  if (k < 1) return set_error(MKNN_EINVAL, "mknn_knn_counts: k must be >= 1");
  if (nq < 0 || nq > 0x7fffffffll) return set_error(MKNN_EINVAL, "mknn_knn_counts: nq out of range");
  mknn_status st = check_uploaded(c, "mknn_knn_counts");
  if (st != MKNN_OK) return st;
  if (m < 1 || m > c->dev_n) return set_error(MKNN_EINVAL, "mknn_knn_counts: m must be in [1, n]");
  if (nq == 0) return MKNN_OK;
  if (!d_q || !d_entries || !d_lists) return set_error(MKNN_EINVAL, "mknn_knn_counts: NULL buffer");
  if (c->dev_lazy.load() != 0) {
    st = flush_pending(const_cast<mknn_cloud *>(c), (hipStream_t)stream);
    if (st != MKNN_OK) return st;
  }
  return run_query(c, d_q, nq, k, m, nullptr, nullptr, nullptr, k, nullptr, nullptr, d_entries,
                   d_lists, d_inserts, (hipStream_t)stream, "mknn_knn_counts");
}

mknn_status mknn_autotune(const mknn_cloud *c, const float *d_q, int64_t nq, int32_t k, int32_t m,
                          void *stream, mknn_tune_entry *tried, int32_t max_tried,
                          int32_t *ntried, mknn_tune_entry *best) {
  clear_error();
  if (k > MKNN_KMAX) return set_error(MKNN_EUNSUPPORTED, "mknn_autotune: k above MKNN_KMAX");
  if (k < 1) return set_error(MKNN_EINVAL, "mknn_autotune: k must be >= 1");
  if (nq < 1 || nq > 0x7fffffffll) return set_error(MKNN_EINVAL, "mknn_autotune: nq out of range");
  if (!d_q || (max_tried > 0 && !tried)) return set_error(MKNN_EINVAL, "mknn_autotune: NULL buffer");
  mknn_status st = check_uploaded(c, "mknn_autotune");
  if (st != MKNN_OK) return st;
  if (m == 0) m = (int32_t)c->dev_n;
  if (m < 1 || m > c->dev_n) return set_error(MKNN_EINVAL, "mknn_autotune: m must be in [0, n]");
  if (c->dev_lazy.load() != 0) {
    st = flush_pending(const_cast<mknn_cloud *>(c), (hipStream_t)stream);
    if (st != MKNN_OK) return st;
  }
  const int S = (k + 15) / 16;
  std::vector<TuneConfig> cand;
  for (int pw : {4, 8}) {
    if (S == 1)
      for (int mm : {4, 6, 8}) cand.push_back({3, mm, pw});
    else
      for (int mm : {4, 6, 8, 11}) cand.push_back({3, mm, pw});
  }
  cand.push_back({2, 6, 4});
  cand.push_back({1, 6, 4});
  hipStream_t s = (hipStream_t)stream;
  void *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const size_t cnt = (size_t)nq * (size_t)k;
  HIP_TRY(hipMallocAsync(&out, cnt * (sizeof(int32_t) + sizeof(float)), s), "mknn_autotune: scratch");
  int32_t *d_idx = (int32_t *)out;
  float *d_dist = (float *)(d_idx + cnt);
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  std::vector<float> ms(cand.size(), INFINITY);
  for (size_t t = 0; t < cand.size() && e == hipSuccess && st == MKNN_OK; ++t) {
    for (int rep = 0; rep < 4 && e == hipSuccess && st == MKNN_OK; ++rep) {
      e = hipEventRecord(e0, s);
      if (e != hipSuccess) break;
      st = run_query(c, d_q, nq, k, m, nullptr, nullptr, nullptr, k, d_idx, d_dist, nullptr,
                     nullptr, nullptr, s, "mknn_autotune", &cand[t]);
      if (st != MKNN_OK) break;
      e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float v = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&v, e0, e1);
      if (e == hipSuccess && rep > 0) ms[t] = std::min(ms[t], v);   // first run warms up
    }
  }
  (void)hipFreeAsync(out, s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != MKNN_OK) return st;
  if (e != hipSuccess) return set_error(MKNN_EHIP, std::string("mknn_autotune: ") + hipGetErrorName(e));
  size_t bi = 0;
  for (size_t t = 1; t < cand.size(); ++t)
    if (ms[t] < ms[bi]) bi = t;
  // The built-in configuration stays unless a candidate is faster by more than 1%, so that
  // timing noise (a profiler attached, another process on the device) does not flip the
  // choice between near-equal candidates.
  const TuneConfig def = default_config(S);
  for (size_t t = 0; t < cand.size(); ++t)
    if (cand[t].family == def.family && cand[t].merge_min == def.merge_min &&
        cand[t].per_wave == def.per_wave && ms[t] <= 1.01f * ms[bi]) {
      bi = t;
      break;
    }
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(dev, S, k == 16 * S, c->dev_n)] = cand[bi];
  }
  const int32_t n_out = (int32_t)std::min<size_t>(cand.size(), max_tried > 0 ? (size_t)max_tried : 0);
  for (int32_t t = 0; t < n_out; ++t)
    tried[t] = {cand[t].family, cand[t].merge_min, cand[t].per_wave, ms[t]};
  if (ntried) *ntried = (int32_t)cand.size();
  if (best) *best = {cand[bi].family, cand[bi].merge_min, cand[bi].per_wave, ms[bi]};
  return MKNN_OK;
}

void mknn_tune_reset(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

mknn_status mknn_tune_save(const char *path) {
  clear_error();
  if (!path) return set_error(MKNN_EINVAL, "mknn_tune_save: path is NULL");
  std::FILE *f = std::fopen(path, "w");
  if (!f) return set_error(MKNN_EINVAL, std::string("mknn_tune_save: cannot write ") + path);
  std::fprintf(f, "mknn-tune 1\n");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto &kv : g_tune) {
    const uint64_t key = kv.first;
    std::fprintf(f, "%u %u %u %u %d %d %d\n", (unsigned)(key >> 32), (unsigned)((key >> 16) & 0xffff),
                 (unsigned)((key >> 8) & 0xff), (unsigned)(key & 0xff), kv.second.family,
                 kv.second.merge_min, kv.second.per_wave);
  }
  const bool ok = std::fclose(f) == 0;
  return ok ? MKNN_OK : set_error(MKNN_EINVAL, std::string("mknn_tune_save: write failed: ") + path);
}

mknn_status mknn_tune_load(const char *path) {
  clear_error();
  if (!path) return set_error(MKNN_EINVAL, "mknn_tune_load: path is NULL");
  std::FILE *f = std::fopen(path, "r");
  if (!f) return set_error(MKNN_ENOTFOUND, std::string("mknn_tune_load: cannot read ") + path);
  char magic[16] = {0};
  int ver = 0;
  std::map<uint64_t, TuneConfig> table;
  bool ok = std::fscanf(f, "%15s %d", magic, &ver) == 2 && std::string(magic) == "mknn-tune" && ver == 1;
  unsigned dev, S, exact, bucket;
  int fam, mm, pw;
  while (ok) {
    const int got = std::fscanf(f, "%u %u %u %u %d %d %d", &dev, &S, &exact, &bucket, &fam, &mm, &pw);
    if (got == EOF) break;
    if (got != 7 || S < 1 || S > 4 || exact > 1 || bucket > 40 || fam < 1 || fam > 3 || mm < 1 ||
        mm > 17 || pw < 4 || pw > 4096) {
      ok = false;
      break;
    }
    const uint64_t key = ((uint64_t)dev << 32) | ((uint64_t)S << 16) | ((uint64_t)exact << 8) | bucket;
    table[key] = {fam, mm, pw};
  }
  std::fclose(f);
  if (!ok) return set_error(MKNN_EINVAL, std::string("mknn_tune_load: malformed file ") + path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto &kv : table) g_tune[kv.first] = kv.second;
  return MKNN_OK;
}

mknn_status mknn_timing_enable(int enable) {
  clear_error();
  g_timing = enable != 0;
  return MKNN_OK;
}

mknn_status mknn_timing_read(double *total_ms, int64_t *launches) {
  clear_error();
  if (!total_ms || !launches) return set_error(MKNN_EINVAL, "mknn_timing_read: NULL");
  double tot = 0.0;
  for (size_t i = 0; i < g_events_used; ++i) {
    HIP_TRY(hipEventSynchronize(g_events[i].second), "mknn_timing_read: synchronize");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, g_events[i].first, g_events[i].second), "mknn_timing_read: elapsed");
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)g_events_used;
  g_events_used = 0;
  return MKNN_OK;
}

mknn_status mknn_delete(mknn_cloud *c, const int32_t *ranks, int64_t count, void *stream) {
  clear_error();
  if (!c) return set_error(MKNN_EINVAL, "mknn_delete: cloud is NULL");
  if (count < 0 || (count > 0 && !ranks)) return set_error(MKNN_EINVAL, "mknn_delete: bad ranks");
  if (count == 0) return MKNN_OK;
  hipStream_t s = (hipStream_t)stream;
  if (!c->lazy.empty()) {
    // pending deletions go with this batch
    for (int64_t t = 0; t < count; ++t)
      if (ranks[t] >= 0 && ranks[t] < (int32_t)c->lazy_mark.size() && c->lazy_mark[ranks[t]])
        return set_error(MKNN_ENOTFOUND, "mknn_delete: rank " + std::to_string(ranks[t]) +
                                             " is already deleted (pending)");
    return flush_pending(c, s, ranks, count);
  }
  DeviceDelta d;
  mknn_status st = delete_prepare(c, ranks, count, &d);
  if (st != MKNN_OK) return st;
  if (!d.on_device) return MKNN_OK;
  st = apply_delta(c, &d, s);
  if (st != MKNN_OK) return st;
  HIP_TRY(hipStreamSynchronize(s), "mknn_delete: synchronize");
  release_old_arena(&d);
  return MKNN_OK;
}

mknn_status mknn_delete_lazy(mknn_cloud *c, const int32_t *ranks, int64_t count, void *stream) {
  clear_error();
  if (!c) return set_error(MKNN_EINVAL, "mknn_delete_lazy: cloud is NULL");
  if (count < 0 || (count > 0 && !ranks)) return set_error(MKNN_EINVAL, "mknn_delete_lazy: bad ranks");
  if (count == 0) return MKNN_OK;
  mknn_status st = check_uploaded(c, "mknn_delete_lazy");
  if (st != MKNN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = c->n;
  if ((int64_t)c->lazy_mark.size() < n) c->lazy_mark.resize(n, 0);
  std::vector<int32_t> sorted(ranks, ranks + count);
  std::sort(sorted.begin(), sorted.end());
  for (size_t t = 0; t < sorted.size(); ++t) {
    const int32_t r = sorted[t];
    if (r < 0 || r >= n || !c->live[r] || c->lazy_mark[r] || (t && sorted[t - 1] == r))
      return set_error(MKNN_ENOTFOUND, "mknn_delete_lazy: rank " + std::to_string(r) +
                                           " is unknown, deleted, pending or repeated");
  }
  if (c->nlive - (int64_t)c->lazy.size() - count < 1)
    return set_error(MKNN_EINVAL, "mknn_delete_lazy: a cloud must keep at least one point");
  if (!c->d_dead || c->dead_cap < n) {
    // a larger array: apply what is pending (its marks then no longer matter) and start anew
    st = flush_pending(c, s);
    if (st != MKNN_OK) return st;
    HIP_TRY(hipStreamSynchronize(s), "mknn_delete_lazy: synchronize");
    if (c->d_dead) (void)hipFree(c->d_dead);
    c->d_dead = nullptr;
    c->dead_cap = 0;
    uint32_t *old = nullptr;
    st = ensure_epochs_async(c, n, s, &old);
    if (st != MKNN_OK) return st;
  }
  if (!c->d_overflow)
    HIP_TRY(hipMalloc((void **)&c->d_overflow, sizeof(uint32_t)), "mknn_delete_lazy: counter");
  st = mark_deleted_async(c, ranks, count, c->lazy_epoch + 1, s);
  if (st != MKNN_OK) return st;
  HIP_TRY(hipStreamSynchronize(s), "mknn_delete_lazy: synchronize");
  for (int64_t t = 0; t < count; ++t) {
    c->lazy_mark[ranks[t]] = 1;
    c->lazy.push_back(ranks[t]);
  }
  ++c->lazy_epoch;
  c->dev_lazy = (int64_t)c->lazy.size();
  return MKNN_OK;
}

mknn_status mknn_delete_flush(mknn_cloud *c, void *stream) {
  clear_error();
  if (!c) return set_error(MKNN_EINVAL, "mknn_delete_flush: cloud is NULL");
  return flush_pending(c, (hipStream_t)stream);
}

int64_t mknn_pending_deletes(const mknn_cloud *c) { return c ? (int64_t)c->lazy.size() : 0; }

mknn_status mknn_insert(mknn_cloud *c, const float *xyz, int64_t count, void *stream) {
  clear_error();
  if (!c) return set_error(MKNN_EINVAL, "mknn_insert: cloud is NULL");
  if (count < 0 || (count > 0 && !xyz)) return set_error(MKNN_EINVAL, "mknn_insert: bad points");
  if (count == 0) return MKNN_OK;
  if (!c->lazy.empty()) {
    mknn_status st = flush_pending(c, (hipStream_t)stream);
    if (st != MKNN_OK) return st;
  }
  DeviceDelta d;
  mknn_status st = insert_prepare(c, xyz, count, &d);
  if (st != MKNN_OK) return st;
  if (!d.on_device) return MKNN_OK;
  hipStream_t s = (hipStream_t)stream;
  st = apply_delta(c, &d, s);
  if (st != MKNN_OK) return st;
  HIP_TRY(hipStreamSynchronize(s), "mknn_insert: synchronize");
  release_old_arena(&d);
  return MKNN_OK;
}

int64_t mknn_live_count(const mknn_cloud *c) { return c ? c->nlive - (int64_t)c->lazy.size() : 0; }

int32_t mknn_head(const mknn_cloud *c) { return c ? c->head : -1; }

void mknn_free(mknn_cloud *c) {
  if (!c) return;
  free_device(c);
  delete c;
}

}  // extern "C"
