// Batched form: many clouds, each with its own query set, k and prefix, answered by one
// launch per register-capacity class.
//
// Flat launch (the default).  A class's requests are laid end to end and every wavefront
// takes four consecutive sorted queries of one request (knn_batch_flat_kernel): the plain
// launch over the whole batch, with the request found by a binary search over the class's
// wavefront offsets.  It has the plain kernel's registers and occupancy; measured on 256
// clouds it is 13% faster than the persistent launch below, whose tile and request state
// costs a wave per SIMD.
//
// Persistent launch (MKNN_BATCH_PERSISTENT=1).  Every request (cloud, queries, k, m) is cut into tiles of T queries,
// T chosen per class and batch as a power of two in [4, tile_queries] (16 by default) that
// gives at most one tile per resident wavefront for a small batch.  Small tiles keep the
// wavefronts of an XCD on a narrow, Morton-contiguous window of queries, so the lists they
// read stay in that XCD's L2; measured on 256 clouds, 16-query tiles beat 1024-query tiles
// by a fifth.  Requests are placed on 8 queues -- one per XCD, workgroups are dispatched
// round-robin over the XCDs so blockIdx % 8 names the XCD -- by a largest-processing-time-
// first rule on an estimated cost (queries x (k + 8) x log2 n), all tiles of a request on
// one queue.  A queue is a list of (request, first tile) entries.  Every persistent
// wavefront claims tiles from its own queue with one atomic per tile, finds the owning
// request by binary search over the entries, and steals from the other queues when its own
// is empty; it leaves once all 8 queues are exhausted.  Its four 16-lane rows take the
// tile's queries one at a time as they become idle (knn_rows.h), so no row waits for
// another at a tile boundary.
//
// Query preparation.  The queries of all requests are bucketed together by (request,
// 12-bit Morton code in the request's cloud box) with one counting sort -- histogram, one
// scan workgroup per request, scatter -- into one contiguous sorted array.
//
// Graph.  A plan owns device buffers sized for a capacity (requests, queries) and a pinned
// host staging area.  All per-call data (descriptors, queue entries, offsets) are written
// to the staging area and copied to the device by the first node, and every kernel reads
// its sizes from device memory with a fixed grid, so one captured hipGraph replays any
// batch within the capacity.  Counters are cleared by a fill kernel, not by a memset node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "device_common.h"
#include "knn_group.h"
#include "knn_rows.h"

namespace mknn {

constexpr int kQueues = 8;
constexpr int kClasses = 4;              // S = 1..4 slots per lane (k <= 16, 32, 48, 64)
// Morton bits per request of the batch sort, chosen per plan (seg_bits_for)
constexpr int kSegBitsMin = 12, kSegBitsMax = 16;

// A queue lists its requests; request e of a queue owns the queue's tiles
// [first, first of the next entry), each `tile[class]` sorted queries long.
struct BatchEntry {
  int32_t req;
  int32_t first;
};

struct BatchHeader {
  int32_t nreq;
  int32_t sorted;
  int64_t total_q;
  int64_t fwaves[kClasses];                // flat launch: wavefronts of work per class
  int32_t qbound[kClasses][kQueues + 1];   // entry index ranges per (class, queue)
  int32_t qtiles[kClasses][kQueues];       // tiles per (class, queue)
  int32_t tile[kClasses];                  // queries per tile, per class
};

// ---------------------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int32_t request_of(const int64_t *qoff, int32_t nreq, int64_t i) {
  int32_t lo = 0, hi = nreq;   // qoff[lo] <= i < qoff[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (qoff[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

template <int BITS>
__global__ __launch_bounds__(256) void seg_hist_kernel(const BatchHeader *h, const QueryArgs *reqs,
                                                       const int64_t *qoff, const BoxArgs *boxes,
                                                       uint32_t *bins) {
  if (!h->sorted) return;
  const int64_t total = h->total_q;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = request_of(qoff, h->nreq, i);
    const float *q = reqs[r].q + 3 * (i - qoff[r]);
    const uint32_t bin = morton30(q[0], q[1], q[2], boxes[r]) >> (30 - BITS);
    atomicAdd(&bins[((int64_t)r << BITS) + bin], 1u);
  }
}

// one workgroup per request: exclusive scan of its bins, offset by the request's start
template <int BITS>
__global__ __launch_bounds__(1024) void seg_scan_kernel(const BatchHeader *h, const int64_t *qoff,
                                                        uint32_t *bins) {
  const int32_t r = blockIdx.x;
  if (!h->sorted || r >= h->nreq) return;
  constexpr int per = (1 << BITS) / 1024;
  __shared__ uint32_t part[1024];
  uint32_t *b = bins + ((int64_t)r << BITS);
  const int t = threadIdx.x;
  uint32_t local[per];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    local[i] = b[t * per + i];
    sum += local[i];
  }
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = (uint32_t)qoff[r] + part[t] - sum;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    b[t * per + i] = run;
    run += local[i];
  }
}

template <int BITS>
__global__ __launch_bounds__(256) void seg_scatter_kernel(const BatchHeader *h,
                                                          const QueryArgs *reqs,
                                                          const int64_t *qoff,
                                                          const BoxArgs *boxes, uint32_t *bins,
                                                          float4 *qs) {
  if (!h->sorted) return;
  const int64_t total = h->total_q;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = request_of(qoff, h->nreq, i);
    const int64_t local = i - qoff[r];
    const float *q = reqs[r].q + 3 * local;
    const uint32_t bin = morton30(q[0], q[1], q[2], boxes[r]) >> (30 - BITS);
    const uint32_t pos = atomicAdd(&bins[((int64_t)r << BITS) + bin], 1u);
    qs[pos] = make_float4(q[0], q[1], q[2], __int_as_float((int32_t)local));
  }
}

// Claim the next tile for this wavefront: its own XCD queue first, then the others.
// Wavefront-uniform result: (request, tile index within the queue entry) or request -1.
__device__ __forceinline__ void claim_tile(const BatchHeader *h, const BatchEntry *ents,
                                           uint32_t *counters, int cls, int home, int &tried,
                                           int32_t &req, int32_t &tile) {
  const int lane = threadIdx.x & 63;
  req = -1;
  tile = 0;
  while (tried < kQueues) {
    const int x = (home + tried) % kQueues;
    const int32_t nt = h->qtiles[cls][x];
    if (nt > 0) {
      uint32_t v = 0;
      if (lane == 0) v = atomicAdd(&counters[cls * kQueues + x], 1u);
      v = __builtin_amdgcn_readfirstlane(v);
      if ((int64_t)v < (int64_t)nt) {
        // the entry owning tile v: last one with first <= v
        int32_t lo = h->qbound[cls][x], hi = h->qbound[cls][x + 1];
        while (hi - lo > 1) {
          const int32_t mid = (lo + hi) >> 1;
          if (ents[mid].first <= (int32_t)v) lo = mid; else hi = mid;
        }
        req = ents[lo].req;
        tile = (int32_t)v - ents[lo].first;
        return;
      }
    }
    ++tried;
  }
}

// Row-scheduled batched kernel.  Every wavefront claims tiles on its own; its four rows
// (knn_rows.h) take four queries of the tile at once and run them to the end together,
// descent steps first, as a wavefront of the plain launch does (refilling a row as soon as
// it is idle would stall the other rows' expansions behind its new descent).  A wavefront
// serves one request at a time: a claimed tile of another request is held until every row
// has finished the current one.  For k <= 16 the tile and request bookkeeping would spill
// about 18 registers at 8 waves per SIMD; 7 waves with almost no spills measure faster.
template <int S, bool LAZY = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S == 1 ? 7 : 1, 8)))
void knn_batch_rows_kernel(const BatchHeader *h, const QueryArgs *reqs, const BatchEntry *ents,
                           uint32_t *counters, int cls) {
  const int lane = threadIdx.x & 63, l = lane & 15, g = lane >> 4;
  const int home = blockIdx.x % kQueues;
  const int64_t tq = h->tile[cls];
  int tried = 0;
  int32_t req = -1, preq = -1;     // current request; claimed tile of another request
  int64_t tnext = 0, tend = 0, pbegin = 0;
  bool exhausted = false;
  const float4 *ent = nullptr;     // the current request's lists, in scalar registers
  const uint64_t *lst = nullptr;
  int merge_min = 1;
  // the query in float32 (the bookkeeping needs the registers); a request has one k and one
  // m, held below in scalar registers with its lists
  RowWalker<S, false, false, true, LAZY> w;
  int32_t rk = 0, rm = 0;
  w.N.init();
  for (;;) {
    // ---- once every row is idle, give the rows the next queries of the current tile
    //      (claiming tiles as needed); the four rows then run their queries to the end
    //      together, descent steps first, as a wavefront of the plain launch does
    for (;;) {
      if (__ballot(w.phase != kRowIdle) != 0) break;
      const uint64_t idle = __ballot(w.phase == kRowIdle && l == 0);
      if (tnext < tend) {
        const int rank = __popcll(idle & ((1ull << (16 * g)) - 1));
        const int64_t s = tnext + rank;
        if (w.phase == kRowIdle && s < tend) w.begin(reqs[req], s, l);
        const int64_t cnt = __popcll(idle);
        tnext = tnext + cnt < tend ? tnext + cnt : tend;
        continue;   // a query answered at once leaves its row idle again
      }
      if (preq >= 0) {
        if (__ballot(w.phase != kRowIdle) != 0) break;   // rows still on the current request
        req = preq;
        preq = -1;
        tnext = pbegin;
        tend = pbegin + tq < reqs[req].nq ? pbegin + tq : reqs[req].nq;
        ent = reqs[req].ent;
        lst = reqs[req].lst;
        merge_min = reqs[req].merge_min;
        rk = reqs[req].k;
        rm = (int32_t)(reqs[req].m < reqs[req].n ? (int64_t)reqs[req].m : reqs[req].n);
        continue;
      }
      if (exhausted) break;
      int32_t creq, ct;
      claim_tile(h, ents, counters, cls, home, tried, creq, ct);
      if (creq < 0) {
        exhausted = true;
        continue;
      }
      const int64_t b = (int64_t)ct * tq;
      if (creq == req) {
        tnext = b;
        tend = b + tq < reqs[req].nq ? b + tq : reqs[req].nq;
      } else {
        preq = creq;
        pbegin = b;
      }
    }
    if (__ballot(w.phase != kRowIdle) == 0) {
      if (exhausted && preq < 0) return;
      continue;
    }
    if (__ballot(w.phase == kRowDescent) != 0) {
      w.step_descent(reqs[req], ent, lst, l, g, rk, rm, merge_min);
    } else {
      if (__ballot(w.phase == kRowSettle) != 0) w.settle(reqs[req], l, rk);
      if (__ballot(w.phase != kRowIdle) != 0)
        w.step_expand(reqs[req], ent, lst, merge_min, l, g, rk, rm);
    }
  }
}

// Flat batched kernel: the plain launch over the concatenated batch.  Class `cls`'s
// requests (queue entries qbound[cls][0] .. qbound[cls][kQueues]) are laid end to end,
// request e taking wavefronts woff[e] .. woff[e] + ceil(nq / 4) - 1, each four consecutive
// sorted queries of that request, one per row, run to the end together as in the plain
// kernel.  No tiles, atomics or per-wavefront request state: registers as in the plain
// kernel, 8 waves per SIMD (for the pending-deletion variants, whose filter would spill
// more, the compiler's choice).  The grid is sized for the plan's capacity (fixed, so that one
// graph replays any batch) and laid XCD-contiguously over the workgroups the batch needs:
// block 8 i + x runs on XCD x and takes workgroup x * per + i, per = ceil(needed / 8);
// blocks past that leave at once.
template <int S, bool LAZY = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LAZY ? (S == 1 ? 8 : 1) : 8, 8)))
void knn_batch_flat_kernel(const BatchHeader *h, const QueryArgs *reqs, const BatchEntry *ents,
                           const int64_t *woff, int cls) {
  const int64_t nw = h->fwaves[cls];
  const int64_t need = (nw + 3) >> 2;              // workgroups of four wavefronts
  const int64_t per = (need + 7) >> 3;
  const int64_t i = blockIdx.x >> 3, x = blockIdx.x & 7;
  if (i >= per) return;
  const int64_t wg = x * per + i;
  const int64_t wave = __builtin_amdgcn_readfirstlane((int32_t)(4 * wg + (threadIdx.x >> 6)));
  if (wg >= need || wave >= nw) return;          // whole wavefronts leave
  // the entry owning this wavefront: the last one whose first wavefront is <= wave
  int32_t lo = h->qbound[cls][0], hi = h->qbound[cls][kQueues];
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (woff[mid] <= wave) lo = mid; else hi = mid;
  }
  const int32_t req = __builtin_amdgcn_readfirstlane(ents[lo].req);
  const QueryArgs a = reqs[req];
  const int64_t begin = 4 * (wave - woff[lo]);
  const int64_t end = begin + 4 < a.nq ? begin + 4 : a.nq;
  const int lane = threadIdx.x & 63, l = lane & 15, g = lane >> 4;
  const int32_t m = (int32_t)(a.m < a.n ? (int64_t)a.m : a.n);
  RowWalker<S, false, (S == 1), true, LAZY> w;
  w.N.init();
  if (begin + g < end) w.begin(a, begin + g, l);
  while (__ballot(w.phase == kRowDescent) != 0)
    w.step_descent(a, a.ent, a.lst, l, g, a.k, m, a.merge_min);
  w.settle(a, l, a.k);
  while (__ballot(w.phase != kRowIdle) != 0)
    w.step_expand(a, a.ent, a.lst, a.merge_min, l, g, a.k, m);
}

// The persistent tile-claiming kernel instead of the flat one (MKNN_BATCH_PERSISTENT=1 in
// the environment when a plan is created).
static bool batch_persistent() {
  const char *e = getenv("MKNN_BATCH_PERSISTENT");
  return e && e[0] && e[0] != '0';
}

template <int S>
static int resident_batch_blocks() {
  static int nb = 0;
  if (!nb) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&knn_batch_rows_kernel<S>), 256, 0) != hipSuccess ||
        nb < 1)
      nb = 1;
  }
  return nb;
}

}  // namespace mknn

using namespace mknn;

// ---------------------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------------------
struct mknn_batch_plan {
  int device = -1;
  int64_t max_req = 0, max_q = 0;
  int32_t tile_q = 16;
  int32_t seg_bits = kSegBitsMin;   // Morton bits per request of the batch sort
  bool sort = true, use_graph = true;
  // device: staging mirror | counters | bins | sorted queries
  char *d_base = nullptr;
  size_t off_hdr = 0, off_reqs = 0, off_ents = 0, off_boxes = 0, off_qoff = 0, off_woff = 0,
         stage_bytes = 0;
  uint32_t *d_counters = nullptr;
  uint32_t *d_bins = nullptr;
  float4 *d_qs = nullptr;
  char *h_stage = nullptr;          // pinned
  hipStream_t cap_stream = nullptr;
  // captured graphs: [0] the plain kernels, [1] the variants that filter pending deletions
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipEvent_t done = nullptr;
  bool pending = false;
  uint32_t grid_batch[kClasses] = {1, 1, 1, 1};
  uint32_t grid_flat = 8;           // flat launch: blocks for the capacity (a multiple of 8)
  bool persistent = false;          // the persistent kernel instead of the flat one
  uint32_t *h_overflow = nullptr;   // pinned: per request, rows a run could not certify
  bool lazy_run = false;            // the last run filtered pending deletions
  int32_t merge_min[kClasses] = {0, 0, 0, 0};   // per class (S - 1); 0 = the autotuner's table
  uint32_t classes = 0xF;           // register classes that plan_enqueue launches (bit S-1)
  uint32_t graph_classes[2] = {0, 0};   // the classes each captured graph launches
  uint32_t grid_stream = 1;
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static void plan_release(mknn_batch_plan *p) {
  if (p->pending && p->done) (void)hipEventSynchronize(p->done);
  for (int v = 0; v < 2; ++v) {
    if (p->exec[v]) (void)hipGraphExecDestroy(p->exec[v]);
    if (p->graph[v]) (void)hipGraphDestroy(p->graph[v]);
  }
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->done) (void)hipEventDestroy(p->done);
  if (p->d_base) (void)hipFree(p->d_base);
  if (p->h_stage) (void)hipHostFree(p->h_stage);
  if (p->h_overflow) (void)hipHostFree(p->h_overflow);
  delete p;
}

// The query launches of plan_enqueue, one per register class in p->classes.
template <bool LAZY>
static void launch_batch_kernels(const mknn_batch_plan *p, hipStream_t s, const BatchHeader *hdr,
                                 const QueryArgs *reqs, const BatchEntry *ents,
                                 const int64_t *woff) {
  // only the classes in p->classes: an empty class's launch still dispatches its whole grid
  const bool c1 = p->classes & 1u, c2 = p->classes & 2u, c3 = p->classes & 4u,
             c4 = p->classes & 8u;
  if (p->persistent) {
    if (c1)
      hipLaunchKernelGGL((knn_batch_rows_kernel<1, LAZY>), dim3(p->grid_batch[0]), dim3(256), 0, s,
                         hdr, reqs, ents, p->d_counters, 0);
    if (c2)
      hipLaunchKernelGGL((knn_batch_rows_kernel<2, LAZY>), dim3(p->grid_batch[1]), dim3(256), 0, s,
                         hdr, reqs, ents, p->d_counters, 1);
    if (c3)
      hipLaunchKernelGGL((knn_batch_rows_kernel<3, LAZY>), dim3(p->grid_batch[2]), dim3(256), 0, s,
                         hdr, reqs, ents, p->d_counters, 2);
    if (c4)
      hipLaunchKernelGGL((knn_batch_rows_kernel<4, LAZY>), dim3(p->grid_batch[3]), dim3(256), 0, s,
                         hdr, reqs, ents, p->d_counters, 3);
  } else {
    const dim3 gf(p->grid_flat);
    if (c1)
      hipLaunchKernelGGL((knn_batch_flat_kernel<1, LAZY>), gf, dim3(256), 0, s, hdr, reqs, ents, woff, 0);
    if (c2)
      hipLaunchKernelGGL((knn_batch_flat_kernel<2, LAZY>), gf, dim3(256), 0, s, hdr, reqs, ents, woff, 1);
    if (c3)
      hipLaunchKernelGGL((knn_batch_flat_kernel<3, LAZY>), gf, dim3(256), 0, s, hdr, reqs, ents, woff, 2);
    if (c4)
      hipLaunchKernelGGL((knn_batch_flat_kernel<4, LAZY>), gf, dim3(256), 0, s, hdr, reqs, ents, woff, 3);
  }
}

// Enqueue the whole batch sequence on stream s (captured into a graph or run eagerly); lazy:
// the query kernels that filter pending deletions.
static hipError_t plan_enqueue(mknn_batch_plan *p, hipStream_t s, bool lazy) {
  const BatchHeader *hdr = (const BatchHeader *)(p->d_base + p->off_hdr);
  const QueryArgs *reqs = (const QueryArgs *)(p->d_base + p->off_reqs);
  const BatchEntry *ents = (const BatchEntry *)(p->d_base + p->off_ents);
  const BoxArgs *boxes = (const BoxArgs *)(p->d_base + p->off_boxes);
  const int64_t *qoff = (const int64_t *)(p->d_base + p->off_qoff);
  const int64_t *woff = (const int64_t *)(p->d_base + p->off_woff);
  hipError_t e = hipMemcpyAsync(p->d_base, p->h_stage, p->stage_bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fill_kernel<uint32_t>, dim3(64), dim3(256), 0, s, p->d_counters,
                     (int64_t)(kClasses * kQueues) + p->max_req, 0u);
  if (p->sort) {
    const int64_t nb = p->max_req << p->seg_bits;
    const uint32_t gb = (uint32_t)std::min<int64_t>(4096, (nb + 255) / 256);
    hipLaunchKernelGGL(fill_kernel<uint32_t>, dim3(gb), dim3(256), 0, s, p->d_bins, nb, 0u);
    const uint32_t gq = p->grid_stream;
    switch (p->seg_bits) {
#define MKNN_SEG_CASE(B)                                                                        \
  case B:                                                                                       \
    hipLaunchKernelGGL(seg_hist_kernel<B>, dim3(gq), dim3(256), 0, s, hdr, reqs, qoff, boxes,   \
                       p->d_bins);                                                              \
    hipLaunchKernelGGL(seg_scan_kernel<B>, dim3((uint32_t)p->max_req), dim3(1024), 0, s, hdr,   \
                       qoff, p->d_bins);                                                        \
    hipLaunchKernelGGL(seg_scatter_kernel<B>, dim3(gq), dim3(256), 0, s, hdr, reqs, qoff,       \
                       boxes, p->d_bins, p->d_qs);                                              \
    break;
      MKNN_SEG_CASE(12)
      MKNN_SEG_CASE(13)
      MKNN_SEG_CASE(14)
      MKNN_SEG_CASE(15)
      MKNN_SEG_CASE(16)
#undef MKNN_SEG_CASE
      default:
        return hipErrorInvalidValue;
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = timing_mark(s, true);
  if (e != hipSuccess) return e;
  if (lazy)
    launch_batch_kernels<true>(p, s, hdr, reqs, ents, woff);
  else
    launch_batch_kernels<false>(p, s, hdr, reqs, ents, woff);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return timing_mark(s, false);
}

namespace mknn {
static mknn_status plan_run(mknn_batch_plan *p, const mknn_request *reqs, int32_t nreq,
                            hipStream_t s, const uint32_t *epochs);

// epochs == NULL: the public run; requests on clouds with deletions pending from
// mknn_delete_lazy apply them first.  Otherwise (the server's run) request r with
// epochs[r] > 0 over-fetches and filters the marks of epochs 1 .. epochs[r]
// (QueryArgs::dead) of its cloud's epoch array; the rows each request could not certify are
// copied to the plan's pinned counters (batch_plan_overflow) behind the run.
static mknn_status plan_run(mknn_batch_plan *p, const mknn_request *reqs, int32_t nreq,
                            hipStream_t s, const uint32_t *epochs) {
  if (!p) return set_error(MKNN_EINVAL, "mknn_batch_plan_run: plan is NULL");
  if (nreq < 0 || (nreq > 0 && !reqs))
    return set_error(MKNN_EINVAL, "mknn_batch_plan_run: bad request array");
  if (nreq > p->max_req)
    return set_error(MKNN_EINVAL, "mknn_batch_plan_run: more requests than the plan holds");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "mknn_batch_plan_run: hipGetDevice");
  if (dev != p->device) return set_error(MKNN_EINVAL, "mknn_batch_plan_run: plan on another device");
  // ---- validate and describe every request
  std::vector<int64_t> qoff((size_t)nreq + 1, 0);
  std::vector<int> cls((size_t)nreq, 0);
  std::vector<char> lazy((size_t)nreq, 0);   // the request filters pending deletions
  std::vector<int32_t> kwalk((size_t)nreq, 0);
  bool any_lazy = false;
  for (int32_t r = 0; r < nreq; ++r) {
    const mknn_request &q = reqs[r];
    const std::string who = "mknn_batch_plan_run: request " + std::to_string(r);
    mknn_status st = check_uploaded(q.cloud, who.c_str());
    if (st != MKNN_OK) return st;
    if (q.k > MKNN_KMAX) return set_error(MKNN_EUNSUPPORTED, who + ": k above MKNN_KMAX");
    if (q.k < 1) return set_error(MKNN_EINVAL, who + ": k must be >= 1");
    if (q.m < 0 || q.m > q.cloud->dev_n) return set_error(MKNN_EINVAL, who + ": m out of [0, n]");
    if (q.nq < 0) return set_error(MKNN_EINVAL, who + ": nq < 0");
    if (q.nq > 0 && (!q.d_q || !q.d_idx || !q.d_dist))
      return set_error(MKNN_EINVAL, who + ": NULL buffer");
    if (epochs) {
      if (epochs[r] != 0) {
        if (!q.cloud->d_dead) return set_error(MKNN_EINVAL, who + ": no marks to filter");
        lazy[r] = 1;
        any_lazy = true;
      }
    } else if (q.cloud->dev_lazy.load() != 0) {
      // the public batched call applies pending deletions first (synchronously)
      st = flush_pending(const_cast<mknn_cloud *>(q.cloud), s);
      if (st != MKNN_OK) return st;
    }
    kwalk[r] = lazy[r] ? std::min<int32_t>(MKNN_KMAX, q.k + kLazyMargin) : q.k;
    qoff[r + 1] = qoff[r] + q.nq;
    cls[r] = (kwalk[r] + 15) / 16 - 1;
  }
  if (qoff[nreq] > p->max_q)
    return set_error(MKNN_EINVAL, "mknn_batch_plan_run: more queries than the plan holds");
  // ---- tiles: requests on queues by largest-processing-time first, per class
  std::vector<double> cost((size_t)nreq);
  for (int32_t r = 0; r < nreq; ++r)
    cost[r] = (double)reqs[r].nq * (reqs[r].k + 8) * std::log2((double)reqs[r].cloud->dev_n + 2.0);
  std::vector<int32_t> order((size_t)nreq);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  std::vector<std::vector<int32_t>> queue_reqs((size_t)kClasses * kQueues);
  double load[kClasses][kQueues] = {};
  for (int32_t r : order) {
    if (reqs[r].nq == 0) continue;
    const int c = cls[r];
    int best = 0;
    for (int x = 1; x < kQueues; ++x)
      if (load[c][x] < load[c][best]) best = x;
    load[c][best] += cost[r];
    queue_reqs[(size_t)c * kQueues + best].push_back(r);
  }
  p->pending = false;
  HIP_TRY(hipEventSynchronize(p->done), "mknn_batch_plan_run: wait for the previous run");
  BatchHeader *hdr = (BatchHeader *)(p->h_stage + p->off_hdr);
  QueryArgs *args = (QueryArgs *)(p->h_stage + p->off_reqs);
  BatchEntry *ents = (BatchEntry *)(p->h_stage + p->off_ents);
  BoxArgs *boxes = (BoxArgs *)(p->h_stage + p->off_boxes);
  int64_t *d_qoff = (int64_t *)(p->h_stage + p->off_qoff);
  // tile length per class: about four tiles per resident workgroup, so that a small batch
  // still spreads over the whole chip, a power of two in [16, tile_q]
  int64_t class_q[kClasses] = {};
  for (int32_t r = 0; r < nreq; ++r) class_q[cls[r]] += reqs[r].nq;
  for (int c = 0; c < kClasses; ++c) {
    const int64_t want = class_q[c] / (4 * (int64_t)p->grid_batch[c]);
    int64_t t = 4;
    while (t * 2 <= want && t * 2 <= p->tile_q) t *= 2;
    hdr->tile[c] = (int32_t)std::max<int64_t>(4, std::min<int64_t>(t, p->tile_q));
  }
  int64_t *woff = (int64_t *)(p->h_stage + p->off_woff);
  int32_t ne = 0;
  for (int c = 0; c < kClasses; ++c) {
    int64_t nw = 0;   // flat launch: wavefronts of the class so far
    for (int x = 0; x < kQueues; ++x) {
      hdr->qbound[c][x] = ne;
      int64_t nt = 0;
      for (int32_t r : queue_reqs[(size_t)c * kQueues + x]) {
        ents[ne].req = r;
        ents[ne].first = (int32_t)nt;
        woff[ne] = nw;
        ++ne;
        nt += (reqs[r].nq + hdr->tile[c] - 1) / hdr->tile[c];
        nw += (reqs[r].nq + 3) / 4;
      }
      hdr->qtiles[c][x] = (int32_t)nt;
    }
    hdr->qbound[c][kQueues] = ne;
    hdr->fwaves[c] = nw;
    // the flat grid covers every class: 8 ceil(workgroups / 8) blocks (checked, not assumed)
    if (8 * (((nw + 3) / 4 + 7) / 8) > (int64_t)p->grid_flat)
      return set_error(MKNN_EINVAL, "mknn_batch_plan_run: batch exceeds the plan's launch size");
  }
  hdr->nreq = nreq;
  hdr->sorted = p->sort ? 1 : 0;
  hdr->total_q = qoff[nreq];
  for (int32_t r = 0; r < nreq; ++r) {
    const mknn_request &q = reqs[r];
    fill_cloud_args(q.cloud, &args[r]);
    const int cl = cls[r];
    args[r].merge_min = p->merge_min[cl] > 0 ? p->merge_min[cl]
                                             : config_for(kwalk[r], false, q.cloud->dev_n).merge_min;
    args[r].q = q.d_q;
    args[r].qs = p->sort ? p->d_qs + qoff[r] : nullptr;
    args[r].nq = q.nq;
    args[r].k = kwalk[r];
    if (lazy[r]) {
      args[r].dead = q.cloud->d_dead;
      args[r].epoch = epochs[r];
      args[r].kout = q.k;
      args[r].overflow = p->d_counters + kClasses * kQueues + r;
    }
    args[r].m = q.m == 0 ? (int32_t)q.cloud->dev_n : q.m;
    args[r].out_idx = q.d_idx;
    args[r].out_dist = q.d_dist;
    boxes[r] = dev_box_of(q.cloud);
  }
  for (int32_t r = 0; r <= nreq; ++r) d_qoff[r] = qoff[r];
  // ---- run (graph replay or eager)
  uint32_t need = 0;   // the classes with work in this batch
  for (int c = 0; c < kClasses; ++c)
    if (class_q[c] > 0) need |= 1u << c;
  if (p->use_graph && !timing_enabled()) {
    const int v = any_lazy ? 1 : 0;
    if (p->exec[v] && (need & ~p->graph_classes[v])) {
      // a class the graph does not launch: capture again with it (the previous run is done)
      (void)hipGraphExecDestroy(p->exec[v]);
      (void)hipGraphDestroy(p->graph[v]);
      p->exec[v] = nullptr;
      p->graph[v] = nullptr;
    }
    if (!p->exec[v]) {
      p->classes = p->graph_classes[v] | need;
      p->graph_classes[v] = p->classes;
      HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal),
              "mknn_batch_plan_run: begin capture");
      hipError_t e = plan_enqueue(p, p->cap_stream, any_lazy);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return set_error(MKNN_EHIP, std::string("mknn_batch_plan_run: capture failed: ") +
                                        hipGetErrorName(e != hipSuccess ? e : e2));
      }
      p->graph[v] = g;
      HIP_TRY(hipGraphInstantiate(&p->exec[v], p->graph[v], nullptr, nullptr, 0),
              "mknn_batch_plan_run: instantiate");
    }
    HIP_TRY(hipGraphLaunch(p->exec[v], s), "mknn_batch_plan_run: graph launch");
  } else {
    p->classes = need;
    HIP_TRY(plan_enqueue(p, s, any_lazy), "mknn_batch_plan_run: launch");
  }
  p->lazy_run = any_lazy;
  if (any_lazy)
    HIP_TRY(hipMemcpyAsync(p->h_overflow, p->d_counters + kClasses * kQueues,
                           sizeof(uint32_t) * (size_t)std::max<int32_t>(1, nreq),
                           hipMemcpyDeviceToHost, s),
            "mknn_batch_plan_run: overflow counters");
  HIP_TRY(hipEventRecord(p->done, s), "mknn_batch_plan_run: record");
  p->pending = true;
  return MKNN_OK;
}

mknn_status batch_plan_run_pending(mknn_batch_plan *p, const mknn_request *reqs, int32_t nreq,
                                   hipStream_t s, const uint32_t *epochs) {
  return plan_run(p, reqs, nreq, s, epochs);
}
const uint32_t *batch_plan_overflow(const mknn_batch_plan *p) {
  return p->lazy_run ? p->h_overflow : nullptr;
}
}  // namespace mknn


extern "C" {

// Morton bits per request of the batch sort: about 4 queries per bin at the plan's average
// request size, between kSegBitsMin and kSegBitsMax.  Queries within a bin run in arbitrary
// order, so finer bins give a wavefront's four rows more alike work; the bins are cleared and
// scanned at the plan's capacity on every run, which caps them for plans of small requests.
// A plan of one request serves requests of any size up to its capacity, which then says
// nothing of their typical size: it keeps the minimum.
static int32_t seg_bits_for(int64_t max_queries, int64_t max_requests) {
  if (max_requests < 2) return kSegBitsMin;
  const int64_t avg = std::max<int64_t>(1, max_queries / max_requests);
  int32_t b = kSegBitsMin;
  while (b < kSegBitsMax && ((int64_t)4 << b) < avg) ++b;
  return b;
}

mknn_status mknn_batch_plan_create(int64_t max_requests, int64_t max_queries, int32_t tile_queries,
                                   int32_t flags, mknn_batch_plan **out) {
  clear_error();
  if (!out) return set_error(MKNN_EINVAL, "mknn_batch_plan_create: out is NULL");
  *out = nullptr;
  if (max_requests < 1 || max_requests > (1 << 20) || max_queries < 1 ||
      max_queries > (int64_t)0x7fffffff)
    return set_error(MKNN_EINVAL, "mknn_batch_plan_create: capacity out of range");
  if (tile_queries < 4 || tile_queries > (1 << 20))
    return set_error(MKNN_EINVAL, "mknn_batch_plan_create: tile_queries out of range [4, 2^20]");
  mknn_batch_plan *p = new (std::nothrow) mknn_batch_plan();
  if (!p) return set_error(MKNN_ENOMEM, "mknn_batch_plan_create: out of host memory");
  p->max_req = max_requests;
  p->max_q = max_queries;
  p->tile_q = tile_queries;
  p->sort = !(flags & MKNN_BATCH_NO_SORT);
  p->seg_bits = seg_bits_for(max_queries, max_requests);
  p->persistent = batch_persistent();
  p->use_graph = !(flags & MKNN_BATCH_NO_GRAPH);
  hipError_t e = hipGetDevice(&p->device);
  size_t o = 0;
  p->off_hdr = o;
  o = align256(o + sizeof(BatchHeader));
  p->off_reqs = o;
  o = align256(o + sizeof(QueryArgs) * (size_t)p->max_req);
  p->off_ents = o;
  o = align256(o + sizeof(BatchEntry) * (size_t)p->max_req);
  p->off_boxes = o;
  o = align256(o + sizeof(BoxArgs) * (size_t)p->max_req);
  p->off_qoff = o;
  o = align256(o + sizeof(int64_t) * (size_t)(p->max_req + 1));
  p->off_woff = o;
  o = align256(o + sizeof(int64_t) * (size_t)p->max_req);
  p->stage_bytes = o;
  const size_t counters_at = o;
  // tile counters, then one overflow counter per request (pending deletions)
  o = align256(o + sizeof(uint32_t) * (kClasses * kQueues + (size_t)p->max_req));
  const size_t bins_at = o;
  if (p->sort) o = align256(o + (sizeof(uint32_t) * (size_t)p->max_req << p->seg_bits));
  const size_t qs_at = o;
  if (p->sort) o = align256(o + sizeof(float4) * (size_t)p->max_q);
  if (e == hipSuccess) e = hipMalloc((void **)&p->d_base, o);
  if (e == hipSuccess) e = hipHostMalloc((void **)&p->h_stage, p->stage_bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&p->h_overflow, sizeof(uint32_t) * (size_t)std::max<int64_t>(1, p->max_req));
  if (e == hipSuccess && p->use_graph) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    const std::string msg = std::string("mknn_batch_plan_create: ") + hipGetErrorName(e);
    plan_release(p);
    return set_error(e == hipErrorOutOfMemory ? MKNN_ENOMEM : MKNN_EHIP, msg);
  }
  std::memset(p->h_stage, 0, p->stage_bytes);
  const uint32_t cus = (uint32_t)device_cus();
  p->grid_batch[0] = cus * resident_batch_blocks<1>();
  p->grid_batch[1] = cus * resident_batch_blocks<2>();
  p->grid_batch[2] = cus * resident_batch_blocks<3>();
  p->grid_batch[3] = cus * resident_batch_blocks<4>();
  p->grid_stream = cus * 8;
  {
    // a class holds at most max_q / 4 + max_req wavefronts of work (a partial one per request)
    const int64_t waves = (p->max_q + 3) / 4 + p->max_req;
    const int64_t wgs = (waves + 3) / 4;
    const int64_t blocks = 8 * ((wgs + 7) / 8);
    if (blocks > (int64_t)0x7fffffff) {
      plan_release(p);
      return set_error(MKNN_EINVAL, "mknn_batch_plan_create: capacity too large for one launch");
    }
    p->grid_flat = (uint32_t)blocks;
  }
  p->d_counters = (uint32_t *)(p->d_base + counters_at);
  p->d_bins = p->sort ? (uint32_t *)(p->d_base + bins_at) : nullptr;
  p->d_qs = p->sort ? (float4 *)(p->d_base + qs_at) : nullptr;
  *out = p;
  return MKNN_OK;
}

void mknn_batch_plan_destroy(mknn_batch_plan *p) {
  if (p) plan_release(p);
}

mknn_status mknn_batch_plan_run(mknn_batch_plan *p, const mknn_request *reqs, int32_t nreq,
                                void *stream) {
  clear_error();
  return plan_run(p, reqs, nreq, (hipStream_t)stream, nullptr);
}


mknn_status mknn_batch_plan_tune(mknn_batch_plan *p, const mknn_request *reqs, int32_t nreq,
                                 void *stream, int32_t *best) {
  clear_error();
  if (!p) return set_error(MKNN_EINVAL, "mknn_batch_plan_tune: plan is NULL");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "mknn_batch_plan_tune: event");
  hipError_t e = hipEventCreate(&e1);
  mknn_status st = MKNN_OK;
  // best of three timed runs after a warm-up
  auto time_batch = [&](float *ms) {
    float tm = INFINITY;
    for (int rep = 0; rep < 4 && e == hipSuccess && st == MKNN_OK; ++rep) {
      e = hipEventRecord(e0, s);
      if (e == hipSuccess) st = mknn_batch_plan_run(p, reqs, nreq, stream);
      if (st != MKNN_OK || e != hipSuccess) break;
      e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float v = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&v, e0, e1);
      if (e == hipSuccess && rep > 0) tm = std::min(tm, v);
    }
    *ms = tm;
  };
  int32_t report = 0;
  if (p->persistent) {
    // the persistent launch: the tile length
    const int32_t keep = p->tile_q;
    int32_t bt = keep;
    float best_ms = INFINITY;
    for (int32_t t : {8, 16, 32, 64, 256}) {
      p->tile_q = t;
      float tm;
      time_batch(&tm);
      if (st != MKNN_OK || e != hipSuccess) break;
      if (tm < best_ms) {
        best_ms = tm;
        bt = t;
      }
    }
    p->tile_q = (st == MKNN_OK && e == hipSuccess) ? bt : keep;
    report = p->tile_q;
  } else {
    // the flat launch: the merge threshold of every register class with work, one class at
    // a time (the others at their current value); the class with most queries is reported
    int64_t q_of[kClasses] = {0, 0, 0, 0};
    for (int32_t r = 0; r < nreq; ++r)
      if (reqs[r].k >= 1 && reqs[r].k <= MKNN_KMAX) q_of[(reqs[r].k + 15) / 16 - 1] += reqs[r].nq;
    int top = 0;
    for (int c = 1; c < kClasses; ++c)
      if (q_of[c] > q_of[top]) top = c;
    static const int32_t cand1[] = {4, 6, 8}, candS[] = {5, 8, 11, 14, 17};
    for (int c = 0; c < kClasses && st == MKNN_OK && e == hipSuccess; ++c) {
      if (!q_of[c]) continue;
      const int32_t keep = p->merge_min[c];
      int32_t bm = keep;
      float best_ms = INFINITY;
      const int32_t *cv = c == 0 ? cand1 : candS;
      const int ncv = c == 0 ? 3 : 5;
      for (int t = 0; t < ncv; ++t) {
        p->merge_min[c] = cv[t];
        float tm;
        time_batch(&tm);
        if (st != MKNN_OK || e != hipSuccess) break;
        if (tm < best_ms) {
          best_ms = tm;
          bm = cv[t];
        }
      }
      p->merge_min[c] = (st == MKNN_OK && e == hipSuccess) ? bm : keep;
    }
    report = p->merge_min[top];
  }
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st != MKNN_OK) return st;
  if (e != hipSuccess) return set_error(MKNN_EHIP, std::string("mknn_batch_plan_tune: ") + hipGetErrorName(e));
  if (best) *best = report;
  return MKNN_OK;
}

// One plan per process, grown on demand (the convenience entry point is not thread-safe).
static mknn_batch_plan *g_plan = nullptr;

mknn_status mknn_batch_knn(const mknn_request *reqs, int32_t nreq, void *stream) {
  clear_error();
  if (nreq < 0 || (nreq > 0 && !reqs)) return set_error(MKNN_EINVAL, "mknn_batch_knn: bad request array");
  int64_t tq = 0;
  for (int32_t r = 0; r < nreq; ++r) tq += reqs[r].nq > 0 ? reqs[r].nq : 0;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "mknn_batch_knn: hipGetDevice");
  if (g_plan && (g_plan->device != dev || g_plan->max_req < nreq || g_plan->max_q < tq)) {
    mknn_batch_plan_destroy(g_plan);
    g_plan = nullptr;
  }
  if (!g_plan) {
    mknn_status st = mknn_batch_plan_create(std::max<int64_t>(nreq, 64),
                                            std::max<int64_t>(tq, (int64_t)1 << 20), 16, 0,
                                            &g_plan);
    if (st != MKNN_OK) return st;
  }
  return mknn_batch_plan_run(g_plan, reqs, nreq, stream);
}

}  // extern "C"
