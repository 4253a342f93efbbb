// Group-per-query variant of the query kernel: 16 lanes (one DPP row) serve one query, four
// queries per 64-wide wavefront.
//
// Why: a list averages ~15 entries.  With 16 lanes a whole list arrives in one coalesced
// 256-byte load, all its distances are computed in parallel, and the descent's "first entry
// closer than the current site" (Alg. 1) is the lowest set bit of a ballot -- one memory
// round trip per list instead of one per entry, and no divergence between entries of a
// list.  The candidate list N (Alg. 2) is spread across the row: lane l holds positions
// S l .. S l + S - 1 (S slots per lane, k <= 16 S).  Inserting a candidate is a row-wide
// compare and a one-position shift, each lane deciding from its own comparisons: inside the
// lane, plus one DPP row move of the lane's last slot into the next lane; only candidates
// that beat the current k-th key are inserted.
//
// Descent and seeding (Alg. 1): when a chunk of L_cur holds an entry closer than the current
// site, only that transition site is offered to N and the walk jumps; a chunk without such
// an entry belongs to the final list of the descent (or to a long list that is about to
// jump later) and all its entries are offered -- the final list doubles as Alg. 2's first
// iteration.  Offering extra true sites to N never changes the result.
//
// Every branch a cross-lane operation depends on is uniform across the 16 lanes of a row.
#pragma once
#include <utility>

#include "knn_kernels.h"

namespace mknn {

__device__ __forceinline__ uint32_t row_bits(uint64_t ballot, int g) {
  return (uint32_t)(ballot >> (16 * g)) & 0xffffu;
}

// (da, ra) < (db, rb) lexicographically; bitwise operators keep it free of branches.
// Squared distances are never negative (nor -0.0, nor NaN), so their IEEE bit patterns
// order like unsigned integers; +inf marks empty slots and compares above every distance.
__device__ __forceinline__ bool key_less(double da, int32_t ra, double db, int32_t rb) {
  const uint64_t ua = (uint64_t)__double_as_longlong(da), ub = (uint64_t)__double_as_longlong(db);
  return (ua < ub) | ((ua == ub) & (ra < rb));
}

// DPP row moves (within each row of 16 lanes):
//   row_shr:1        lane l reads lane l-1 (lane 0 keeps `old`)
//   row_newbcast:15  every lane reads lane 15 of its row
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowBcast15 = 0x15F;
constexpr int kDppRowBcast0 = 0x150;    // row_newbcast:0, every lane reads lane 0 of its row

// Every use below either has a valid source lane for every lane or ignores the lanes that
// do not (row_shr:1 at lane 0), so the DPP move needs no "old" operand (bound_ctrl).
template <int CTRL>
__device__ __forceinline__ int32_t dpp_i32(int32_t /*unused*/, int32_t x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xf, 0xf, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double old, double x) {
  const int64_t o = __double_as_longlong(old), v = __double_as_longlong(x);
  const int32_t lo = dpp_i32<CTRL>((int32_t)o, (int32_t)v);
  const int32_t hi = dpp_i32<CTRL>((int32_t)(o >> 32), (int32_t)(v >> 32));
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Partner lanes of the compare-exchange stages (lane l ^ X within a row of 16).
template <int X>
__device__ __forceinline__ int32_t xor_lane(int32_t x) {
  if constexpr (X == 1) return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xf, 0xf, true);    // quad_perm 1,0,3,2
  if constexpr (X == 2) return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xf, 0xf, true);    // quad_perm 2,3,0,1
  if constexpr (X == 3) return __builtin_amdgcn_mov_dpp(x, 0x1B, 0xf, 0xf, true);    // quad_perm 3,2,1,0
  if constexpr (X == 4) return __builtin_amdgcn_ds_swizzle(x, 0x101F);               // bitmask mode, xor 4
  if constexpr (X == 7) return __builtin_amdgcn_mov_dpp(x, 0x141, 0xf, 0xf, true);   // row_half_mirror
  if constexpr (X == 8) return __builtin_amdgcn_mov_dpp(x, 0x128, 0xf, 0xf, true);   // row_ror:8
  if constexpr (X == 15) return __builtin_amdgcn_mov_dpp(x, 0x140, 0xf, 0xf, true);  // row_mirror
  return x;
}

template <int X>
__device__ __forceinline__ double xor_lane_f64(double x) {
  const int64_t v = __double_as_longlong(x);
  const int32_t lo = xor_lane<X>((int32_t)v), hi = xor_lane<X>((int32_t)(v >> 32));
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// One compare-exchange stage between lanes l and l ^ X: of each pair, the lane whose bit
// BIT is clear keeps the smaller key, the other the larger.  Equal keys only occur between
// identical padding entries.
template <int X, int BIT>
__device__ __forceinline__ void cas_stage(double &d, int32_t &r, int l) {
  const double pd = xor_lane_f64<X>(d);
  const int32_t pr = xor_lane<X>(r);
  const bool take = key_less(pd, pr, d, r) == ((l & BIT) == 0);
  d = take ? pd : d;
  r = take ? pr : r;
}

// Ascending bitonic sort of one key per lane across the row.  Each merge level starts by
// comparing mirrored lanes (l ^ 3, l ^ 7, l ^ 15), so that every stage keeps the minimum in
// the lower lane of a pair and only four lane masks are needed.
__device__ __forceinline__ void row_sort16(double &d, int32_t &r, int l) {
  cas_stage<1, 1>(d, r, l);
  cas_stage<3, 2>(d, r, l);
  cas_stage<1, 1>(d, r, l);
  cas_stage<7, 4>(d, r, l);
  cas_stage<2, 2>(d, r, l);
  cas_stage<1, 1>(d, r, l);
  cas_stage<15, 8>(d, r, l);
  cas_stage<4, 4>(d, r, l);
  cas_stage<2, 2>(d, r, l);
  cas_stage<1, 1>(d, r, l);
}

// Whether v equals any lane's x in the row: row_ror:t for t = 1..15 passes every value of
// the row by every lane once.
template <int T>
__device__ __forceinline__ int32_t row_ror(int32_t x) {
  if constexpr (T == 0) return x;
  else return __builtin_amdgcn_mov_dpp(x, 0x120 + T, 0xf, 0xf, true);
}
template <int... T>
__device__ __forceinline__ bool in_row(int32_t v, int32_t x, std::integer_sequence<int, T...>) {
  return ((v == row_ror<T>(x)) | ...);
}

// Lanes of one wavefront exchanging values through LDS.  The hardware completes a
// wavefront's LDS operations in program order, but the compiler must be told that other
// lanes write the memory between two phases: otherwise it may forward a lane's own earlier
// store to a later load of the same address.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-row LDS of the row kernels, S > 1 (16 rows of a 256-thread workgroup).  A row's ring
// of transition sites (written by the descent, read once by settle) and its merge area
// (expansion only) are never in use at the same time, so they share the row's bytes.  The
// row size is 16 words more than a multiple of 32, so the two rows of a 32-lane LDS pass
// fall on different banks.
template <int S>
struct RowLds {
  static constexpr int L = 16 * S, W = L + 16;
  union {
    struct {
      double d[L];
      int32_t r[L];
    } ring;
    struct {
      double nd[L];     // position p at (p mod S) 16 + p / S
      int32_t nr[W];
      uint32_t m[W];
    } merge;
  };
  int32_t pad[16];
};
template <int S>
__device__ __forceinline__ RowLds<S> &row_lds() {
  __shared__ RowLds<S> rows[16];
  return rows[threadIdx.x >> 4];
}

template <int S, bool EXACTK>
struct RowTopK {
  double d[S];
  int32_t r[S];
  double thr_d;    // key of slot k-1 (uniform in the row)
  int32_t thr_r;

  __device__ __forceinline__ void init() {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      d[s] = INFINITY;
      r[s] = kEmpty;
    }
    thr_d = INFINITY;
    thr_r = kEmpty;
  }

  // Recompute the threshold (key of slot k-1) after N was written directly.
  __device__ __forceinline__ void refresh_threshold(int k) {
    if (EXACTK) {
      thr_d = dpp_f64<kDppRowBcast15>(d[S - 1], d[S - 1]);
      thr_r = dpp_i32<kDppRowBcast15>(r[S - 1], r[S - 1]);
    } else {
      slot(k - 1, thr_d, thr_r);
    }
  }

  // position j (row-uniform) broadcast to the row: slot j % S of lane j / S
  __device__ __forceinline__ void slot(int j, double &od, int32_t &orr) const {
    const uint32_t s = (uint32_t)j % S, src = (uint32_t)j / S;
    double vd = d[0];
    int32_t vr = r[0];
#pragma unroll
    for (int t = 1; t < S; ++t) {
      vd = ((uint32_t)t == s) ? d[t] : vd;
      vr = ((uint32_t)t == s) ? r[t] : vr;
    }
    od = __shfl(vd, (int)src, 16);
    orr = __shfl(vr, (int)src, 16);
  }

  // Insert the row-uniform candidate (cd, cr) unless already present.  Only called for a
  // candidate that beats the current k-th key.  Returns 1 if inserted.
  __device__ __forceinline__ int insert(double cd, int32_t cr, int l, int g, int k) {
    if (!place(cd, cr, l, g)) return 0;
    refresh_threshold(k);
    return 1;
  }

  // Shift the row-uniform candidate (cd, cr) into the sorted slots unless the row already
  // holds its rank; the threshold is left as it was.  A candidate that ranks past the last
  // slot changes nothing.  Returns false if the rank was held.
  __device__ __forceinline__ bool place(double cd, int32_t cr, int l, int g) {
    bool has = false;
#pragma unroll
    for (int s = 0; s < S; ++s) has |= (r[s] == cr);
    if (row_bits(__ballot(has), g)) return false;
    // Every lane decides from its own comparisons: a position whose key is below the
    // candidate keeps it; the first one that is not (its predecessor is below, or it is
    // position 0) takes the candidate; every later one takes its predecessor's key.  The
    // predecessor of slot 0 is the last slot of lane l - 1 (DPP row_shr:1); lane 0 reads 0
    // there (no source lane), which stands for "below".
    bool lt[S];
#pragma unroll
    for (int s = 0; s < S; ++s) lt[s] = key_less(d[s], r[s], cd, cr);
    const int32_t prev_above =
        __builtin_amdgcn_update_dpp(0, lt[S - 1] ? 0 : 1, kDppRowShr1, 0xf, 0xf, true);
    const double pd = dpp_f64<kDppRowShr1>(d[S - 1], d[S - 1]);
    const int32_t pr = dpp_i32<kDppRowShr1>(r[S - 1], r[S - 1]);
#pragma unroll
    for (int s = S - 1; s >= 0; --s) {
      const bool prev_lt = s > 0 ? lt[s > 0 ? s - 1 : 0] : prev_above == 0;
      const double prevd = s > 0 ? d[s > 0 ? s - 1 : 0] : pd;
      const int32_t prevr = s > 0 ? r[s > 0 ? s - 1 : 0] : pr;
      d[s] = lt[s] ? d[s] : (prev_lt ? cd : prevd);
      r[s] = lt[s] ? r[s] : (prev_lt ? cr : prevr);
    }
    return true;
  }

  // k <= 16 (one slot per lane): merge every lane's candidate with `better` set at once.
  // Candidates already in N are dropped, the rest are sorted by a bitonic network; the
  // elementwise minimum of the ascending N and the mirrored (descending) candidates is
  // bitonic and holds the 16 smallest keys of both, and a bitonic merge sorts it.  Fixed
  // cost, no per-candidate control flow, so the four rows of a wavefront run it together.
  __device__ __forceinline__ int merge16(bool better, double dd, int32_t rr, int l, int k) {
    static_assert(S == 1, "merge16 serves one slot per lane");
    // evaluated by every lane: the row moves must see all 16 ranks of N
    const bool dup = in_row(rr, r[0], std::make_integer_sequence<int, 16>{});
    better = better & !dup;
    double cd = better ? dd : INFINITY;
    int32_t cr = better ? rr : kEmpty;
    row_sort16(cd, cr, l);
    cd = xor_lane_f64<15>(cd);
    cr = xor_lane<15>(cr);
    const bool cm = key_less(cd, cr, d[0], r[0]);
    d[0] = cm ? cd : d[0];
    r[0] = cm ? cr : r[0];
    cas_stage<8, 8>(d[0], r[0], l);
    cas_stage<4, 4>(d[0], r[0], l);
    cas_stage<2, 2>(d[0], r[0], l);
    cas_stage<1, 1>(d[0], r[0], l);
    if (EXACTK) {
      thr_d = dpp_f64<kDppRowBcast15>(d[0], d[0]);
      thr_r = dpp_i32<kDppRowBcast15>(r[0], r[0]);
    } else {
      slot(k - 1, thr_d, thr_r);
    }
    return better ? 1 : 0;
  }

  // k > 16 (S slots per lane, lane l holding positions S l .. S l + S - 1): merge every
  // lane's candidate with `better` set at once, by ranks.  The candidates are sorted across
  // the row and each finds by binary search over N (staged in LDS) how many keys of N lie
  // below it, p; a candidate whose rank N already holds meets its own key there and is
  // dropped.  The kept ones, numbered 0, 1, ... in order, have non-decreasing p, so the
  // number of kept candidates below the key at position i is the largest (number + 1) of a
  // kept candidate with p <= i: each kept candidate posts (number + 1) at position p with
  // an LDS maximum, and a running maximum over the positions (within the lane, then across
  // the row by DPP) gives every key its count.  Every key's new position is its old one
  // plus that count; the keys that land below 16 S are scattered back into the staging
  // area (every search has read it by then) and read back.  Position p is held in LDS at
  // (p mod S) 16 + p / S, and the 4-byte rows are padded, against bank conflicts.  Kept candidates and keys of N
  // never tie (equal keys mean equal ranks), so the new positions are a permutation.  The
  // LDS areas are per row (16 rows of a 256-thread workgroup); the lanes of a row exchange
  // values through them without a barrier, as LDS operations of one wavefront complete in
  // program order.
  __device__ __forceinline__ int mergeS(bool better, double dd, int32_t rr, int l, int g,
                                        int k) {
    static_assert(S > 1, "mergeS serves more than one slot per lane");
    constexpr int L = 16 * S;
    constexpr int TOP = S == 2 ? 32 : 64;   // a power of two >= L / 2 (S = 2, 3, 4)
    // position p is stored at (p mod S) 16 + p / S: each slot's 16 positions are contiguous,
    // so staging and reading back a lane's slots are free of bank conflicts
    // (unsigned: S = 2 and 4 then take a mask and a shift, S = 3 a multiply-high)
    auto at = [](uint32_t p) { return (p % S) * 16u + p / S; };
    RowLds<S> &lds = row_lds<S>();
    double *s_nd = lds.merge.nd;
    int32_t *s_nr = lds.merge.nr;
    uint32_t *s_m = lds.merge.m;
    double cd = better ? dd : INFINITY;
    int32_t cr = better ? rr : kEmpty;
    row_sort16(cd, cr, l);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      s_nd[16 * s + l] = d[s];
      s_nr[16 * s + l] = r[s];
      s_m[16 * s + l] = 0u;
    }
    wave_lds_sync();
    // keys of N below the candidate (binary lifting over the sorted L keys)
    uint32_t p = 0;
#pragma unroll
    for (int step = TOP; step > 0; step >>= 1)
      if (p + step <= L &&
          key_less(s_nd[at(p + step - 1)], s_nr[at(p + step - 1)], cd, cr))
        p += step;
    const bool real = cr != kEmpty;
    const bool held = real && p < L && s_nr[at(p < L ? p : 0)] == cr;
    const bool kept = real && !held;
    const uint32_t jk = __popc(row_bits(__ballot(kept), g) & ((1u << l) - 1u));
    if (kept && p < L) atomicMax(&s_m[at(p)], jk + 1u);
    wave_lds_sync();
    // kept candidates below each key: running maximum within the lane, then the maximum
    // over the lanes below (inclusive scan by DPP row_shr, shifted by one lane)
    uint32_t below[S];
    uint32_t run = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      run = max(run, s_m[16 * s + l]);
      below[s] = run;
    }
    uint32_t sc = run;
    sc = max(sc, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)sc, 0x111, 0xf, 0xf, false));
    sc = max(sc, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)sc, 0x112, 0xf, 0xf, false));
    sc = max(sc, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)sc, 0x114, 0xf, 0xf, false));
    sc = max(sc, (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)sc, 0x118, 0xf, 0xf, false));
    const uint32_t lower = (uint32_t)__builtin_amdgcn_update_dpp(0, (int32_t)sc, 0x111, 0xf, 0xf, false);
    if (kept && jk + p < L) {   // every lane's searches read the staged keys before this
      s_nd[at(jk + p)] = cd;
      s_nr[at(jk + p)] = cr;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t np = (uint32_t)(S * l + s) + max(lower, below[s]);
      if (np < L) {
        s_nd[at(np)] = d[s];
        s_nr[at(np)] = r[s];
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < S; ++s) {
      d[s] = s_nd[16 * s + l];
      r[s] = s_nr[16 * s + l];
    }
    if (EXACTK) {
      thr_d = dpp_f64<kDppRowBcast15>(d[S - 1], d[S - 1]);
      thr_r = dpp_i32<kDppRowBcast15>(r[S - 1], r[S - 1]);
    } else {
      slot(k - 1, thr_d, thr_r);
    }
    return better ? 1 : 0;
  }

  // k <= 16 (one slot per lane): insert the flagged candidates of each row one by one, in
  // lane order, and refresh the threshold once at the end.  A candidate is not tested
  // against the threshold again after each insertion: one that no longer ranks compares
  // above every slot and changes nothing.  Per candidate, slot l keeps its key if that key
  // is smaller (or the row already holds the candidate's rank), takes the candidate if it
  // is the first slot that does not, and otherwise takes slot l-1's key (DPP row_shr:1).
  __device__ __forceinline__ void insert_each16(bool cand, double dd, int32_t rr, int l, int g,
                                                int k) {
    static_assert(S == 1, "insert_each16 serves one slot per lane");
    uint32_t mask = row_bits(__ballot(cand), g);   // uniform in the row
    while (mask) {
      const int j = __ffs(mask) - 1;
      mask &= mask - 1u;
      const double cd = __shfl(dd, j, 16);
      const int32_t cr = __shfl(rr, j, 16);
      const bool held = row_bits(__ballot(r[0] == cr), g) != 0;
      const bool keep = held || key_less(d[0], r[0], cd, cr);
      // lane l-1's "moved" flag; lane 0 reads 0 (no source lane: either DPP bound mode
      // leaves or writes 0)
      const int32_t prev_moved =
          __builtin_amdgcn_update_dpp(0, keep ? 0 : 1, kDppRowShr1, 0xf, 0xf, true);
      const double pd = dpp_f64<kDppRowShr1>(d[0], d[0]);
      const int32_t pr = dpp_i32<kDppRowShr1>(r[0], r[0]);
      const bool take = prev_moved == 0;
      d[0] = keep ? d[0] : (take ? cd : pd);
      r[0] = keep ? r[0] : (take ? cr : pr);
    }
    refresh_threshold(k);
  }

  // k > 16 (S slots per lane): insert the flagged candidates of each row one by one, in
  // lane order, and refresh the threshold once at the end (slot k-1 takes a cross-lane read
  // when k < 16 S).  A candidate is not tested against the threshold again after each
  // insertion: one that no longer ranks lands past the last slot and changes nothing.
  __device__ __forceinline__ void insert_each(bool cand, double dd, int32_t rr, int l, int g,
                                              int k) {
    uint32_t mask = row_bits(__ballot(cand), g);   // uniform in the row
    while (mask) {
      const int j = __ffs(mask) - 1;
      mask &= mask - 1u;
      place(__shfl(dd, j, 16), __shfl(rr, j, 16), l, g);
    }
    refresh_threshold(k);
  }

  // Offer every lane's (dd, rr) with `better` set; updates the threshold as it goes.
  __device__ __forceinline__ int insert_all(bool better, double dd, int32_t rr, int l, int g,
                                            int k) {
    int ins = 0;
    uint32_t mask = row_bits(__ballot(better), g);
    while (mask) {
      const int j = __ffs(mask) - 1;
      const double cd = __shfl(dd, j, 16);
      const int32_t cr = __shfl(rr, j, 16);
      ins += insert(cd, cr, l, g, k);
      better = better && l != j && key_less(dd, rr, thr_d, thr_r);
      mask = row_bits(__ballot(better), g);
    }
    return ins;
  }
};

struct ScanState {
  int32_t nent = 0, nins = 0;
};

// Scan one list chunk by chunk.  DESCENT: stop at the first entry strictly closer than the
// current site and jump to it.  Returns true if the descent jumped.
template <int S, bool EXACTK, bool DESCENT, bool COUNT>
__device__ __forceinline__ bool scan_list(const QueryArgs &a, RowTopK<S, EXACTK> &N,
                                          uint64_t dsc, double qx, double qy, double qz,
                                          int32_t m, int k, int l, int g, int32_t &cur,
                                          double &dcur, ScanState &cs) {
  const uint32_t st = (uint32_t)dsc, len = (uint32_t)(dsc >> 32);
  for (uint32_t base = 0; base < len; base += 16) {
    const uint32_t e = base + (uint32_t)l;
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    if (e < len) c = a.ent[st + e];
    const int32_t r = __float_as_int(c.w);
    const bool valid = e < len && r < m;
    double dd = INFINITY;
    if (valid) {
      const double dx = qx - (double)c.x, dy = qy - (double)c.y, dz = qz - (double)c.z;
      dd = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    }
    const uint32_t vmask = row_bits(__ballot(valid), g);
    if (DESCENT) {
      const uint32_t jm = row_bits(__ballot(valid && dd < dcur), g);
      if (jm) {
        const int j = __ffs(jm) - 1;
        if (COUNT) cs.nent += j + 1;
        dcur = __shfl(dd, j, 16);
        cur = __shfl(r, j, 16);
        // the transition site joins N (Alg. 1); entries before it were not closer
        if (key_less(dcur, cur, N.thr_d, N.thr_r)) {
          const int ins = N.insert(dcur, cur, l, g, k);
          if (COUNT) cs.nins += ins;
        }
        return true;
      }
    }
    if (COUNT) cs.nent += __popc(vmask);
    const bool better = valid && key_less(dd, r, N.thr_d, N.thr_r);
    int ins = 0;
    if constexpr (S == 1) {
      // the most candidates any row of the wavefront has in this chunk (wave-uniform)
      const uint64_t wb = __ballot(better);
      const int most = max(max(__popc((uint32_t)wb & 0xffffu), __popc((uint32_t)(wb >> 16) & 0xffffu)),
                           max(__popc((uint32_t)(wb >> 32) & 0xffffu), __popc((uint32_t)(wb >> 48))));
      if (most > 0 && most >= a.merge_min) {
        const int got = N.merge16(better, dd, r, l, k);
        if (COUNT) ins = __popc(row_bits(__ballot(got), g));
      } else if (most > 0) {
        ins = N.insert_all(better, dd, r, l, g, k);
      }
    } else {
      ins = N.insert_all(better, dd, r, l, g, k);
    }
    if (COUNT) cs.nins += ins;
    if (vmask != 0xffffu) break;   // end of the list or of the prefix
  }
  return false;
}

// One query (sorted position s of request a) on one 16-lane row.  Row-uniform control.
template <int S, bool EXACTK, bool COUNT>
__device__ __forceinline__ void group_query(const QueryArgs &a, int64_t s, int l, int g) {
  double qx, qy, qz;
  int64_t qi;
  if (a.qs) {
    const float4 v = a.qs[s];
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
  if (k < 1 || k > 16 * S || m < 1) return;

  RowTopK<S, EXACTK> N;
  N.init();
  ScanState cs;
  int32_t nlist = 0;
  if (a.head < m) {
    // ---- Alg. 1: descent from the head
    int32_t cur = a.head;
    double dcur;
    {
      const double dx = qx - (double)a.hx, dy = qy - (double)a.hy, dz = qz - (double)a.hz;
      dcur = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    }
    if (l == 0) {
      N.d[0] = dcur;
      N.r[0] = cur;
    }
    if (k == 1) {
      N.thr_d = dcur;
      N.thr_r = cur;
    }
    for (;;) {
      if (COUNT) ++nlist;
      if (!scan_list<S, EXACTK, true, COUNT>(a, N, a.lst[cur], qx, qy, qz, m, k, l, g, cur,
                                             dcur, cs))
        break;
    }
    // ---- Alg. 2: expand the lists of the confirmed neighbours N[2..k-1] (1-based)
    for (int i = 1; i < k - 1; ++i) {
      double pd;
      int32_t pr;
      N.slot(i, pd, pr);
      if (pr == kEmpty) break;
      if (COUNT) ++nlist;
      int32_t dummy_c = 0;
      double dummy_d = 0.0;
      scan_list<S, EXACTK, false, COUNT>(a, N, a.lst[pr], qx, qy, qz, m, k, l, g, dummy_c,
                                         dummy_d, cs);
    }
  }
  if (COUNT) {
    if (l == 0) {
      a.cnt_entries[qi] = cs.nent;
      a.cnt_lists[qi] = nlist;
      if (a.cnt_inserts) a.cnt_inserts[qi] = cs.nins;
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const int j = S * l + t;   // lane l holds positions S l .. S l + S - 1
    if (j < k) {
      const bool empty = N.r[t] == kEmpty;
      a.out_idx[row + j] = empty ? -1 : N.r[t];
      a.out_dist[row + j] = empty ? INFINITY : (float)sqrt(N.d[t]);
    }
  }
}

// Plain launch: one row per query, queries in (sorted) order, XCD-contiguous tiles.
// Eight wavefronts per SIMD (the hardware maximum) hide most of the walk's memory latency.
// For one slot per lane the merge network's lane masks would otherwise take enough scalar
// registers to cost one; wider candidate lists are left to the compiler (forcing eight
// would spill vector registers).
template <int S, bool EXACTK, bool COUNT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S == 1 ? 8 : 1, 8))) void knn_group_kernel(QueryArgs a) {
  const int lane = threadIdx.x & 63;
  const int l = lane & 15, g = lane >> 4;
  const int64_t wave =
      ((int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t s = wave * 4 + g;
  if (s >= a.nq) return;            // whole rows leave together
  group_query<S, EXACTK, COUNT>(a, s, l, g);
}

}  // namespace mknn
