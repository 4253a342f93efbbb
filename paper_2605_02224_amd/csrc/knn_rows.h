// Row-scheduled variant of the group kernel: the same 16-lane rows and candidate list as
// knn_group.h, but every row advances through its own queries independently.
//
// Why: in the group kernel the four rows of a wavefront run one query each from start to
// end, so a row whose descent (Alg. 1) or list is shorter waits, masked off, for the
// longest one; about half of all lane-cycles were spent masked.  Here each step processes
// one 16-entry chunk for every row -- a descent chunk, an expansion chunk (Alg. 2) or the
// next chunk of a long list -- so a row in its descent and a row in its expansion run the
// same instructions, and a row that finishes writes its result and takes another query
// while the others go on.  Candidate insertion is shared: the chunk's candidates of all
// four rows go through one merge network (or the one-by-one insertion) together.
//
// Per chunk the row state decides what the chunk means:
//   descent   : the first entry closer than the current site is the transition site; it
//               is offered to N and the walk jumps to its list.  A list without one is the
//               final list of the descent, offered whole (it doubles as Alg. 2's first
//               iteration, exactly as in the group kernel).
//   expansion : every entry of the list of N's slot `it` whose key lies above that slot's
//               key is offered (it = 1 .. k-2); the nearer ones are already in N.
#pragma once
#include <type_traits>

#include "knn_group.h"

namespace mknn {

// Offer every lane's flagged candidate to N, the four rows at once.
template <int S, bool EXACTK>
__device__ __forceinline__ void offer_all(RowTopK<S, EXACTK> &N, bool cand, double dd,
                                          int32_t rr, int l, int g, int k, int merge_min) {
  const uint64_t wb = __ballot(cand);
  if (wb == 0) return;
  const int most = max(max(__popc((uint32_t)wb & 0xffffu), __popc((uint32_t)(wb >> 16) & 0xffffu)),
                       max(__popc((uint32_t)(wb >> 32) & 0xffffu), __popc((uint32_t)(wb >> 48))));
  if (most >= merge_min) {
    if constexpr (S == 1)
      N.merge16(cand, dd, rr, l, k);
    else
      N.mergeS(cand, dd, rr, l, g, k);
    return;
  }
  if constexpr (S == 1)
    N.insert_each16(cand, dd, rr, l, g, k);
  else
    N.insert_each(cand, dd, rr, l, g, k);
}

// kRowSettle (descent steps first): the descent has ended and N is still to be seeded from
// the ring (settle()).
constexpr int32_t kRowDescent = 0, kRowExpand = 1, kRowIdle = 2, kRowSettle = 3;

// Per-row rings of transition sites, 16 S entries (the class's largest k) for each of the
// 16 rows of a 256-thread workgroup (every launch of these kernels uses 256 threads).  In
// LDS rather than registers: 32 more VGPRs per lane would cost occupancy.  For S > 1 the
// ring shares the row's LDS with the merge area (RowLds).
__shared__ double g_ring1_d[16 * 16];
__shared__ int32_t g_ring1_r[16 * 16];
template <int S>
__device__ __forceinline__ double *ring_d() {
  if constexpr (S == 1) return g_ring1_d + 16 * (threadIdx.x >> 4);
  else return row_lds<S>().ring.d;
}
template <int S>
__device__ __forceinline__ int32_t *ring_r() {
  if constexpr (S == 1) return g_ring1_r + 16 * (threadIdx.x >> 4);
  else return row_lds<S>().ring.r;
}

// Entry idx of a list: the record {x, y, z, rank} (the layout of every query launch), or,
// for the measurement of the layout choice only: kLayoutRanks, its rank from the ranks-only
// array and then the point from the rank-indexed point array, a dependent 16-byte gather;
// kLayoutArrays, its rank and its three coordinates from four arrays of 4-byte values.
// in_list: the lane's entry lies inside the list (the padding past a list holds no rank).
template <int LAYOUT>
__device__ __forceinline__ float4 load_entry(const QueryArgs &a, const float4 *ent, uint32_t idx,
                                             bool in_list) {
  if constexpr (LAYOUT == kLayoutRecords) {
    (void)a;
    (void)in_list;
    return ent[idx];
  } else if constexpr (LAYOUT == kLayoutRanks) {
    (void)ent;
    const int32_t r = a.rk[idx];
    float4 p = a.pts[in_list ? r : 0];
    p.w = __int_as_float(in_list ? r : kEmpty);
    return p;
  } else {
    (void)ent;
    (void)in_list;
    return make_float4(a.sx[idx], a.sy[idx], a.sz[idx], __int_as_float(a.rk[idx]));
  }
}

// The state of one row's current query.  Row-uniform values, held by every lane of the row.
// WIDE_Q: hold the query in float64 (widened once rather than at every chunk), where the
// registers allow it.  UNIFORM: one k and one m for the whole launch (or, batched, for the
// request the wavefront is on) -- no per-query arrays, and k and m stay scalars.  LAZY: the
// launch may filter pending deletions (QueryArgs::dead); kept out of the other launches,
// whose registers (and so occupancy) the filter would cost.
template <int S, bool EXACTK, bool WIDE_Q = (S == 1), bool UNIFORM = EXACTK, bool LAZY = false,
          int LAYOUT = kLayoutRecords>
struct RowWalker {
  RowTopK<S, EXACTK> N;
  using QCoord = typename std::conditional<WIDE_Q, double, float>::type;
  QCoord qx = 0, qy = 0, qz = 0;   // the query
  double dcur = 0;
  int32_t qi = 0;                  // caller index of the query (nq < 2^31)
  int32_t k = 0, m = 0, cur = 0, it = 0;
  int32_t phase = kRowIdle;
  uint64_t dsc = 0;
  uint32_t base = 0;
  // key of the confirmed neighbour whose list an expansion row scans (slot `it` of N)
  double od = 0;
  int32_t orr = 0;
  // Descent steps first: the transition sites of the descent (Alg. 1) go to a ring of 16 S
  // in LDS (entry t % 16 S for the t-th); each is strictly closer than the one before, so
  // the last k are the only ones that can rank among the k nearest and the ring holds them
  // sorted.
  int32_t ntrans = 0;

  // Start the query at sorted position s of request a.  A query whose prefix holds no live
  // site is answered at once (empty row) and leaves the row idle.
  __device__ __forceinline__ void begin(const QueryArgs &a, int64_t s, int l) {
    phase = kRowIdle;
    dsc = 0;   // an idle row reads record 0 of whatever arena the wavefront is on
    base = 0;
    if (a.qs) {
      const float4 v = a.qs[s];
      qx = v.x;
      qy = v.y;
      qz = v.z;
      qi = __float_as_int(v.w);
    } else {
      qi = (int32_t)s;
      qx = a.q[3 * s];
      qy = a.q[3 * s + 1];
      qz = a.q[3 * s + 2];
    }
    k = !UNIFORM && a.kq ? a.kq[qi] : a.k;
    // pending deletions: walk for more neighbours than the row keeps (at most the class's)
    if constexpr (LAZY && !UNIFORM)
      if (a.kq && a.dead) k = k + kLazyMargin < 16 * S ? k + kLazyMargin : 16 * S;
    int64_t mm = !UNIFORM && a.mq ? (int64_t)a.mq[qi] : (int64_t)a.m;
    if (mm > a.n) mm = a.n;
    m = (int32_t)mm;
    if (k < 1 || k > 16 * S || m < 1) return;
    N.init();
    if (a.head >= m) {
      finish(a, l, k);
      return;
    }
    cur = a.head;
    const double dx = (double)qx - (double)a.hx, dy = (double)qy - (double)a.hy,
                 dz = (double)qz - (double)a.hz;
    dcur = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    if (l == 0) {
      ring_d<S>()[0] = dcur;
      ring_r<S>()[0] = cur;
    }
    ntrans = 1;
    if constexpr (S > 1) {
      // the step<false> path seeds N with the transition sites directly
      if (l == 0) {
        N.d[0] = dcur;
        N.r[0] = cur;
      }
      if (k == 1) {
        N.thr_d = dcur;
        N.thr_r = cur;
      }
    }
    dsc = a.lst[cur];
    base = 0;
    it = 0;
    phase = kRowDescent;
  }

  // uk: the launch's (request's) k when UNIFORM, held by the caller in a scalar register
  __device__ __forceinline__ void finish(const QueryArgs &a, int l, int32_t uk) {
    const int32_t k = EXACTK ? 16 * S : (UNIFORM ? uk : this->k);
    if constexpr (LAZY) {
      if (a.dead) {
        finish_live(a, l, k);
        return;
      }
    }
    const int64_t row = !UNIFORM && a.row_off ? a.row_off[qi] : qi * (int64_t)k;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int j = S * l + t;   // lane l holds positions S l .. S l + S - 1
      if (j < k) {
        const bool empty = N.r[t] == kEmpty;
        a.out_idx[row + j] = empty ? -1 : N.r[t];
        a.out_dist[row + j] = empty ? INFINITY : (float)sqrt(N.d[t]);
      }
    }
    phase = kRowIdle;
    dsc = 0;
    base = 0;
  }

  // Pending deletions: N holds the k nearest listed sites, marked ones included.  The row
  // keeps the first kout unmarked ones, in order; these are the kout nearest remaining sites
  // whenever N holds that many (every remaining site not in N is farther than all of N).  A
  // row with fewer is exact only if N is not full (then N holds every site of the prefix);
  // otherwise it is padded and counted in *overflow, and its caller answers it again once
  // the deletions are applied.  Row-uniform control; the row's lanes are all active.
  __device__ __forceinline__ void finish_live(const QueryArgs &a, int l, int32_t k) {
    const int g = (int)((threadIdx.x & 63) >> 4);
    const int32_t ko = !UNIFORM && a.kq ? a.kq[qi] : a.kout;
    const int64_t row = !UNIFORM && a.row_off ? a.row_off[qi] : qi * (int64_t)ko;
    // position S l + t (lane l holds S consecutive positions): the unmarked entries before
    // it are those of the lanes below l, and those of this lane's earlier slots
    bool live[S];
    int32_t before = 0, kept = 0;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int32_t r = N.r[t];
      const bool listed = S * l + t < k && r != kEmpty;
      uint32_t e = 0;
      if (listed) e = a.dead[r];
      live[t] = listed && (e == 0 || e > a.epoch);
      const uint32_t lm = row_bits(__ballot(live[t]), g);
      before += __popc(lm & ((1u << l) - 1u));
      kept += __popc(lm);
    }
#pragma unroll
    for (int t = 0; t < S; ++t) {
      if (live[t] && before < ko) {
        a.out_idx[row + before] = N.r[t];
        a.out_dist[row + before] = (float)sqrt(N.d[t]);
      }
      before += live[t] ? 1 : 0;
    }
    for (int32_t j = kept + l; j < ko; j += 16) {
      a.out_idx[row + j] = -1;
      a.out_dist[row + j] = INFINITY;
    }
    if (kept < ko) {
      double ld;
      int32_t lr;
      N.slot(k - 1, ld, lr);
      if (lr != kEmpty && l == 0) atomicAdd(a.overflow, 1u);
    }
    phase = kRowIdle;
    dsc = 0;
    base = 0;
  }

  // One chunk for every row of the wavefront (call from uniform control flow).  A row that
  // completes its query writes the result (through `a`) and becomes idle.  The list arrays
  // come in separately so that callers can keep them in scalar registers.
  //
  // DESCENT_FIRST: while any row of the wavefront is in its descent, the rows in their
  // expansion wait.  Descent chunks are cheap (no candidate step for k <= 16), and the
  // candidate step then runs when all rows have candidates to offer.  Worth it only when
  // every row holds one query for the whole launch; rows refilled with new queries would
  // stall the others' expansions at every refill.
  template <bool DESCENT_FIRST>
  // uk, um (UNIFORM): the launch's (request's) k and m clamped to n, in scalar registers.
  __device__ __forceinline__ void step(const QueryArgs &a, const float4 *ent,
                                       const uint64_t *lst, int merge_min, int l, int g,
                                       int32_t uk, int32_t um) {
    // uniform launches: k and m are the same for every row, so they stay scalars
    const int32_t k = EXACTK ? 16 * S : (UNIFORM ? uk : this->k);
    const int32_t m = UNIFORM ? um : this->m;
    const bool any_descent = DESCENT_FIRST && __ballot(phase == kRowDescent) != 0;
    const bool active = any_descent ? phase == kRowDescent : phase != kRowIdle;
    const uint32_t st = (uint32_t)dsc, len = (uint32_t)(dsc >> 32);
    const uint32_t e = base + (uint32_t)l;
    // every lane loads, without a branch: a chunk never reaches more than 15 records past
    // the end of a list (or of the arena's used part), which the arena's padding covers;
    // records past the list are ignored.  An idle row's descriptor is 0 (begin and finish
    // reset it), so it never points into another request's arena in the batched form.
    const float4 c = load_entry<LAYOUT>(a, ent, st + e, e < len);
    const int32_t r = __float_as_int(c.w);
    const bool valid = active && e < len && r < m;
    const double dx = (double)qx - (double)c.x, dy = (double)qy - (double)c.y,
                 dz = (double)qz - (double)c.z;
    const double dv = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    const double dd = valid ? dv : INFINITY;
    const uint32_t vmask = row_bits(__ballot(valid), g);
    const uint32_t jm = row_bits(__ballot(valid && phase == kRowDescent && dd < dcur), g);
    const int j = jm ? __ffs(jm) - 1 : 0;
    // k <= 16: descent rows offer nothing (their transition sites go to the ring and the
    // final list is scanned again as the first expansion).  Otherwise a jumping row offers
    // its transition site only (Alg. 1) and the other rows every entry.
    // An expansion row scans the list of slot `it`, and slots 0 .. it are final by then
    // (Theorem 1: each further neighbour is a transition site or in the list of a nearer
    // one, all of whose lists came first), so an entry whose key is not above slot it's
    // is already in N and is not offered.
    bool cand;
    if constexpr (S == 1)
      cand = valid && phase == kRowExpand && key_less(od, orr, dd, r) &&
             key_less(dd, r, N.thr_d, N.thr_r);
    else
      cand = (jm ? l == j : valid) && (phase != kRowExpand || key_less(od, orr, dd, r)) &&
             key_less(dd, r, N.thr_d, N.thr_r);
    offer_all(N, cand, dd, r, l, g, k, merge_min);
    if (jm) {
      dcur = __shfl(dd, j, 16);
      cur = __shfl(r, j, 16);
      if constexpr (S == 1) {
        if (l == (ntrans & 15)) {
          ring_d<1>()[l] = dcur;
          ring_r<1>()[l] = cur;
        }
        ++ntrans;
      }
      dsc = lst[cur];
      base = 0;
    } else if (S == 1 && active && phase == kRowDescent &&
               !(vmask == 0xffffu && base + 16 < len)) {
      // the descent ends at p_cur: N starts as the last transition sites, nearest first,
      // and the final list is scanned again as the expansion of N[0]
      const int have = ntrans < 16 ? ntrans : 16;
      const int src = (ntrans - 1 - l) & 15;
      N.d[0] = l < have ? ring_d<S>()[src] : INFINITY;
      N.r[0] = l < have ? ring_r<S>()[src] : kEmpty;
      N.refresh_threshold(k);
      od = dcur;   // slot 0: the nearest site, p_cur
      orr = cur;
      if (k == 1) {
        finish(a, l, k);
      } else {
        phase = kRowExpand;
        it = 0;
        base = 0;
      }
    } else if (active) {
      if (vmask == 0xffffu && base + 16 < len) {
        base += 16;   // the next chunk of a long list
      } else {
        // the list is finished: the next confirmed neighbour's list, or the query is done
        it = phase == kRowDescent ? 1 : it + 1;
        phase = kRowExpand;
        int32_t pr = kEmpty;
        double pd = 0;
        if (it < k - 1) N.slot(it, pd, pr);
        if (pr != kEmpty) {
          od = pd;
          orr = pr;
          dsc = lst[pr];
          base = 0;
        } else {
          finish(a, l, k);
        }
      }
    }
  }

  // Descent steps first (DESCENT_FIRST): the two kinds of step below do what step<true>
  // does, each with only the work its rows need.  While some row of the wavefront is in its
  // descent only those rows advance, offering nothing to N: the transition sites go to the
  // ring.  Once no row is, settle() seeds N from the ring and every busy row expands; the
  // descent's final list is scanned again as the expansion of N[0], p_cur.

  // A step while some row is in its descent.
  __device__ __forceinline__ void step_descent(const QueryArgs &a, const float4 *ent,
                                               const uint64_t *lst, int l, int g, int32_t uk,
                                               int32_t um, int merge_min = 0) {
    (void)uk;
    (void)merge_min;
    const int32_t m = UNIFORM ? um : this->m;
    const bool desc = phase == kRowDescent;
    const uint32_t st = (uint32_t)dsc, len = (uint32_t)(dsc >> 32);
    const uint32_t e = base + (uint32_t)l;
    const float4 c = load_entry<LAYOUT>(a, ent, st + e, e < len);   // in bounds for every lane: see step()
    const int32_t r = __float_as_int(c.w);
    const bool valid = desc && e < len && r < m;
    const double dx = (double)qx - (double)c.x, dy = (double)qy - (double)c.y,
                 dz = (double)qz - (double)c.z;
    const double dv = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    const uint32_t vmask = row_bits(__ballot(valid), g);
    const uint32_t jm = row_bits(__ballot(valid && dv < dcur), g);
    if (jm) {
      // the first strictly closer entry is the next transition site (Alg. 1)
      const int j = __ffs(jm) - 1;
      dcur = __shfl(dv, j, 16);
      cur = __shfl(r, j, 16);
      if (l == (ntrans & 15)) {
        ring_d<S>()[(uint32_t)ntrans % (16u * S)] = dcur;
        ring_r<S>()[(uint32_t)ntrans % (16u * S)] = cur;
      }
      ++ntrans;
      dsc = lst[cur];
      base = 0;
    } else if (desc) {
      if (vmask == 0xffffu && base + 16 < len)
        base += 16;   // the next chunk of a long list
      else
        phase = kRowSettle;   // the descent ends at p_cur; N is seeded by settle()
    }
  }

  // A row whose descent has ended at p_cur starts N as the last transition sites, nearest
  // first, and scans the final list again as the expansion of N[0].  Called once no row is
  // in its descent (kept out of the descent steps, whose loop then carries fewer values).
  // Position S l + t of N takes the (S l + t)-th newest site of the ring.
  __device__ __forceinline__ void settle(const QueryArgs &a, int l, int32_t uk) {
    const int32_t k = EXACTK ? 16 * S : (UNIFORM ? uk : this->k);
    wave_lds_sync();   // the ring entries were written by other lanes of the row
    if (phase != kRowSettle) return;
    constexpr int R = 16 * S;
    const int have = ntrans < R ? ntrans : R;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int pos = S * l + t;
      const int src = pos < have ? (int)((uint32_t)(ntrans - 1 - pos) % (uint32_t)R) : 0;
      N.d[t] = pos < have ? ring_d<S>()[src] : INFINITY;
      N.r[t] = pos < have ? ring_r<S>()[src] : kEmpty;
    }
    N.refresh_threshold(k);
    od = dcur;
    orr = cur;
    if (k == 1) {
      finish(a, l, k);
    } else {
      phase = kRowExpand;
      it = 0;
      base = 0;
    }
  }

  // A step while no row is in its descent: every busy row scans a chunk of the list of N's
  // slot `it` and offers the entries above that slot's key and not above the k-th key.  The
  // two tests compare D only: an entry tied in D with the owner but of smaller rank is
  // already in N, and one tied with the k-th key but of larger rank lands past the last
  // slot, so offering them changes nothing.
  __device__ __forceinline__ void step_expand(const QueryArgs &a, const float4 *ent,
                                              const uint64_t *lst, int merge_min, int l, int g,
                                              int32_t uk, int32_t um) {
    const int32_t k = EXACTK ? 16 * S : (UNIFORM ? uk : this->k);
    const int32_t m = UNIFORM ? um : this->m;
    const bool act = phase != kRowIdle;
    const uint32_t st = (uint32_t)dsc, len = (uint32_t)(dsc >> 32);
    const uint32_t e = base + (uint32_t)l;
    const float4 c = load_entry<LAYOUT>(a, ent, st + e, e < len);
    const int32_t r = __float_as_int(c.w);
    const bool valid = act && e < len && r < m;
    const double dx = (double)qx - (double)c.x, dy = (double)qy - (double)c.y,
                 dz = (double)qz - (double)c.z;
    const double dv = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    const uint32_t vmask = row_bits(__ballot(valid), g);
    const bool cand = valid && dv >= od && dv <= N.thr_d;
    offer_all(N, cand, dv, r, l, g, k, merge_min);
    if (act) {
      if (vmask == 0xffffu && base + 16 < len)
        base += 16;
      else
        next_list(a, lst, l, k, it + 1);
    }
  }

  // Expand the list of N's slot `nit` next, or finish the query when there is none.
  __device__ __forceinline__ void next_list(const QueryArgs &a, const uint64_t *lst, int l,
                                            int32_t k, int32_t nit) {
    it = nit;
    phase = kRowExpand;
    int32_t pr = kEmpty;
    double pd = 0;
    if (it < k - 1) N.slot(it, pd, pr);
    if (pr != kEmpty) {
      od = pd;
      orr = pr;
      dsc = lst[pr];
      base = 0;
    } else {
      finish(a, l, k);
    }
  }
};

// Plain launch: a wavefront owns `per_wave` consecutive sorted queries; row g takes
// positions g, g + 4, g + 8, ... of them, so the rows stay on Morton neighbours.  Eight
// waves per SIMD for every class: the wider candidate lists then spill a few registers
// (S = 4: 16), which costs less than the latency fewer waves leave exposed.
template <int S, bool EXACTK, bool DESCENT_FIRST, bool UNIFORM, bool LAZY = false>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(8, 8)))
void knn_rows_kernel(QueryArgs a, int32_t per_wave) {
  const int lane = threadIdx.x & 63;
  const int l = lane & 15, g = lane >> 4;
  const int64_t wave =
      ((int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t begin = wave * per_wave;
  const int64_t end = begin + per_wave < a.nq ? begin + per_wave : a.nq;
  RowWalker<S, EXACTK, (S == 1), UNIFORM, LAZY> w;
  w.N.init();
  const int32_t m = (int32_t)(a.m < a.n ? (int64_t)a.m : a.n);
  if constexpr (DESCENT_FIRST) {
    // 4 queries per wavefront: each row takes its one query and runs it to the end
    if (begin + g < end) w.begin(a, begin + g, l);
    while (__ballot(w.phase == kRowDescent) != 0)
      w.step_descent(a, a.ent, a.lst, l, g, a.k, m, a.merge_min);
    w.settle(a, l, a.k);
    while (__ballot(w.phase != kRowIdle) != 0)
      w.step_expand(a, a.ent, a.lst, a.merge_min, l, g, a.k, m);
  } else {
    int64_t next = begin + g;
    for (;;) {
      while (w.phase == kRowIdle && next < end) {
        w.begin(a, next, l);
        next += 4;
      }
      if (__ballot(w.phase != kRowIdle) == 0) break;
      w.template step<false>(a, a.ent, a.lst, a.merge_min, l, g, a.k, m);
    }
  }
}

// The row kernel over another layout of the lists (k == 16, one k and m per launch, descent
// steps first): the measurement of what the records' layout saves.  Same walk and results as
// knn_rows_kernel<1, true, true, true>.
template <int LAYOUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8)))
void knn_rows_layout_kernel(QueryArgs a, int32_t per_wave) {
  static_assert(LAYOUT == kLayoutRanks || LAYOUT == kLayoutArrays, "a layout to measure");
  const int lane = threadIdx.x & 63;
  const int l = lane & 15, g = lane >> 4;
  const int64_t wave =
      ((int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t begin = wave * per_wave;
  const int64_t end = begin + per_wave < a.nq ? begin + per_wave : a.nq;
  RowWalker<1, true, true, true, false, LAYOUT> w;
  w.N.init();
  const int32_t m = (int32_t)(a.m < a.n ? (int64_t)a.m : a.n);
  if (begin + g < end) w.begin(a, begin + g, l);
  while (__ballot(w.phase == kRowDescent) != 0)
    w.step_descent(a, a.ent, a.lst, l, g, a.k, m, a.merge_min);
  w.settle(a, l, a.k);
  while (__ballot(w.phase != kRowIdle) != 0)
    w.step_expand(a, a.ent, a.lst, a.merge_min, l, g, a.k, m);
}

}  // namespace mknn
