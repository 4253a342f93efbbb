// Query kernels for gfx950: the 1-NN descent of Alg. 1 fused with the k-expansion of
// Alg. 2, one query per lane, over successor lists resident in HBM.
//
// Device layout of one cloud:
//   ent[]  16-byte records {x, y, z, rank} (float, float, float, int32 bit pattern).  The
//          entries of list L_i are contiguous and ascending in rank (Sec. 3); whole lists
//          are placed in the Morton order of their owner points.  The array is padded with
//          kEntPad records so a 16-lane chunk may reach 15 records past the end of a list.
//   lst[r] 64-bit descriptor: start index of L_r in ent (low 32 bits) | length (high 32).
// Each list entry carries its point's coordinates, so scanning a list is one contiguous
// read and no second gather is needed to evaluate the distance.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mknn {

constexpr int kEntPad = 16;
constexpr int32_t kEmpty = 0x7fffffff;   // rank of an empty candidate slot

struct QueryArgs {
  const float4 *ent;
  const uint64_t *lst;
  float hx, hy, hz;          // coordinates of the head (oldest live site)
  int32_t head;
  int64_t n;
  const float *q;            // [nq][3] in caller order
  const float4 *qs;          // sorted queries {x, y, z, original index} or NULL
  int64_t nq;
  int32_t k, m;              // scalars (used when kq / mq are NULL)
  const int32_t *kq, *mq;    // per-query k and m (caller order) or NULL
  const int64_t *row_off;    // ragged rows (with kq) or NULL
  int32_t *out_idx;
  float *out_dist;
  int32_t *cnt_entries, *cnt_lists;   // diagnostics (COUNT variant only)
  int32_t *cnt_inserts;               // optional diagnostic: candidates inserted into N
  int32_t merge_min;                  // k <= 16: candidates per chunk from which a merge
                                      // network replaces one-by-one insertion (0 = default)
  // Pending (lazy) deletions: dead[r] is the epoch (1, 2, ...) of the deletion batch that
  // marked rank r, 0 if none.  The ranks marked in epochs 1 .. epoch are still listed but no
  // longer part of this call's cloud (later epochs are deletions it must not see).  The walk
  // then runs for more neighbours than asked (k, or per query kq + kLazyMargin) and a row
  // keeps the first kout (per query: kq) not so marked; a row whose walk filled all its
  // slots with fewer than kout such sites cannot be certified and counts itself in
  // *overflow.  dead == NULL: no pending deletions.
  const uint32_t *dead;
  uint32_t epoch;
  int32_t kout;
  uint32_t *overflow;
  // Other layouts of the same lists, for the measurement that compares them with the
  // records above (only the layout kernel reads these): rk[i] is the rank of record i;
  // ranks only: pts[r] is the point of rank r; four arrays: sx, sy, sz[i] are the
  // coordinates of record i.
  const int32_t *rk = nullptr;
  const float4 *pts = nullptr;
  const float *sx = nullptr, *sy = nullptr, *sz = nullptr;
};

// List layouts of the layout measurement (the query launches use kLayoutRecords).
constexpr int kLayoutRecords = 0, kLayoutRanks = 1, kLayoutArrays = 2;

// Extra neighbours a walk collects per query while deletions are pending.
constexpr int32_t kLazyMargin = 16;

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range
// of tiles so Morton-adjacent queries share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb) {
  uint32_t x = b & 7u, i = b >> 3, q8 = nb >> 3, r8 = nb & 7u;
  return x * q8 + (x < r8 ? x : r8) + i;
}

// Squared distance exactly as the brute-force definition: float64 from float32 inputs,
// every operation rounded, no fused multiply-add.
__device__ __forceinline__ double sq_dist(double qx, double qy, double qz, float4 c) {
  const double dx = qx - (double)c.x;
  const double dy = qy - (double)c.y;
  const double dz = qz - (double)c.z;
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

}  // namespace mknn
