// Successor lists built on the GPU (the construction of Sec. 3, computed in parallel).
//
// The lists record, for every rank j, its Delaunay neighbours in DT(P_{1:j}) (Sec. 3, Fig. 2
// caption).  Those neighbours are the finite vertices of the tetrahedra that the insertion of
// p_j creates in the sequential incremental construction, and which tetrahedra that is does
// not depend on the order the work is done in: a tetrahedron t with vertex set D(t) and
// conflict set C(t) (the later sites inside its circumsphere, or beyond its hull facet for a
// ghost) is created by the sequential construction exactly when every site of D(t) is older
// than every site of C(t), and it is created by the newest site of D(t).  So every created
// tetrahedron can be generated from ridges (shared triangles), in rounds, with no global
// order (the ridge formulation of randomized incremental Delaunay construction by Blelloch,
// Gu, Shun and Sun, "Parallelism in randomized incremental algorithms"):
//
//   for a ridge r shared by tetrahedra t1 and t2 with c1 = min C(t1) < c2 = min C(t2):
//   site c1 destroys t1 but not t2, so r lies on the boundary of c1's cavity and c1 creates
//   t = (r, c1), whose conflict set is the part of C(t1) u C(t2) in conflict with t.  Then
//   r is shared by t and t2 (processed again in the next round), and each of t's three
//   ridges through c1 is shared with another tetrahedron created by c1: whichever of the
//   two arrives second at that ridge (a hash table on the ridge's vertices) emits the pair.
//   A ridge with c1 == c2 is inside one cavity (or final, when both are empty): dropped.
//
// Every (finite ridge vertex i, c1) of a created tetrahedron is a list entry (i, c1); the
// entries are sorted and made unique into the CSR lists.  The predicates are the
// construction's own: the site being tested is always newer than the tetrahedron's
// vertices, so "conflict" is the sequential test (inside or on the circumsphere; a ghost:
// strictly beyond its facet, or in its plane inside or on its circumcircle).  The device
// evaluates them in float64 with the forward error bounds of the host predicates and
// defers every sign it cannot certify to the host, which decides it exactly; so the lists
// equal the sequential construction's, entry for entry, degenerate inputs included.
//
// Work per round, all on the stream given: classify the ridge pairs; prefix sums give the
// new tetrahedra and a flat range of candidate tests; one thread per candidate tests it;
// deferred tests are decided on the host; a prefix sum over the accepted candidates packs
// the new conflict lists; the new tetrahedra check in their ridges.  Sites are positions in
// the insertion order (a rank in the ordinary case).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <array>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "cloud.h"
#include "exact.h"

namespace mknn {
namespace gbuild {

constexpr int32_t kNone = INT32_MAX;       // empty conflict set
constexpr uint64_t kEmptyKey = ~0ull;
constexpr int32_t kEmptyVal = -1;
constexpr int kSiteBits = 21;              // ridge keys pack three site ids of 21 bits
constexpr int64_t kMaxSites = ((int64_t)1 << kSiteBits) - 2;
constexpr int kMaxProbes = 1 << 16;        // a ridge table slot is found long before this
// error bits a kernel sets instead of going on
constexpr uint32_t kErrRidge = 1;          // a ridge pair that does not share a triangle
constexpr uint32_t kErrTable = 2;          // the ridge table has no free slot near a key

struct Item {          // one ridge pair, and what classifying it decided
  int32_t t1, t2;
};
struct Job {           // a tetrahedron being created, or an initial one being filled
  int32_t tnew;        // its id
  int32_t td;          // the tetrahedron destroyed (its list is read first)
  int32_t ts;          // the survivor across the ridge (-1: none)
  int32_t p;           // the creating site (-1: none)
  int32_t nd;          // candidates taken from td's list (the rest come from ts's)
  int32_t apex;        // index of p among tnew's vertices (-1: none)
};
struct Deferred {      // a candidate test whose sign the device could not certify
  int32_t v[4];        // the new tetrahedron
  int32_t vd[4];       // the destroyed one (used when the candidate comes from ts)
  int32_t q;
  int32_t from_td;
  int64_t idx;         // candidate index
  int32_t tnew;        // the new tetrahedron's id (its min conflict takes q if accepted)
  int32_t pad;
};

__device__ __forceinline__ double3 site(const float4 *P, int32_t v) {
  const float4 f = P[v];
  return make_double3((double)f.x, (double)f.y, (double)f.z);
}

// The double evaluations and error bounds of the host predicates; 0 = not certified.
__device__ __forceinline__ int orient_filter(double3 a, double3 b, double3 c, double3 d) {
  const double bx = b.x - a.x, by = b.y - a.y, bz = b.z - a.z;
  const double cx = c.x - a.x, cy = c.y - a.y, cz = c.z - a.z;
  const double dx = d.x - a.x, dy = d.y - a.y, dz = d.z - a.z;
  const double m0 = cy * dz - cz * dy;
  const double m1 = cx * dz - cz * dx;
  const double m2 = cx * dy - cy * dx;
  const double det = bx * m0 - by * m1 + bz * m2;
  const double perm = fabs(bx) * (fabs(cy * dz) + fabs(cz * dy)) +
                      fabs(by) * (fabs(cx * dz) + fabs(cz * dx)) +
                      fabs(bz) * (fabs(cx * dy) + fabs(cy * dx));
  const double bound = kOrientBound * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return 0;
}

// +1: e strictly inside the sphere of the positively oriented (a,b,c,d); -1: strictly
// outside; 0: not certified.
__device__ __forceinline__ int insphere_filter(double3 a, double3 b, double3 c, double3 d,
                                               double3 e) {
  double r[4][3], L[4];
  const double3 pts[4] = {a, b, c, d};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r[i][0] = pts[i].x - e.x;
    r[i][1] = pts[i].y - e.y;
    r[i][2] = pts[i].z - e.z;
    L[i] = r[i][0] * r[i][0] + r[i][1] * r[i][1] + r[i][2] * r[i][2];
  }
  auto m3 = [&](int i, int j, int k, double &perm) {
    const double m0 = r[j][1] * r[k][2] - r[j][2] * r[k][1];
    const double m1 = r[j][0] * r[k][2] - r[j][2] * r[k][0];
    const double m2 = r[j][0] * r[k][1] - r[j][1] * r[k][0];
    perm = fabs(r[i][0]) * (fabs(r[j][1] * r[k][2]) + fabs(r[j][2] * r[k][1])) +
           fabs(r[i][1]) * (fabs(r[j][0] * r[k][2]) + fabs(r[j][2] * r[k][0])) +
           fabs(r[i][2]) * (fabs(r[j][0] * r[k][1]) + fabs(r[j][1] * r[k][0]));
    return r[i][0] * m0 - r[i][1] * m1 + r[i][2] * m2;
  };
  double p0, p1, p2, p3;
  const double M0 = m3(1, 2, 3, p0), M1 = m3(0, 2, 3, p1), M2 = m3(0, 1, 3, p2),
               M3 = m3(0, 1, 2, p3);
  const double det = (L[1] * M1 - L[0] * M0) + (L[3] * M3 - L[2] * M2);
  const double perm = L[0] * p0 + L[1] * p1 + L[2] * p2 + L[3] * p3;
  const double bound = kInsphereBound * perm;
  if (det > bound) return -1;
  if (-det > bound) return 1;
  return 0;
}

// Conflict of site q (newer than every vertex) with tetrahedron v: 1 yes, 0 no, 2 not
// certified (the host decides; this includes every exact tie).
__device__ __forceinline__ int conflict_filter(const float4 *P, const int4 v, double3 q) {
  const int32_t w[4] = {v.x, v.y, v.z, v.w};
  int inf = -1;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (w[i] < 0) inf = i;
  double3 x[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) x[i] = (w[i] < 0) ? q : site(P, w[i]);
  if (inf < 0) {
    const int s = insphere_filter(x[0], x[1], x[2], x[3], q);
    return s > 0 ? 1 : (s < 0 ? 0 : 2);
  }
  const int o = orient_filter(x[0], x[1], x[2], x[3]);
  return o > 0 ? 1 : (o < 0 ? 0 : 2);
}

__device__ __forceinline__ uint64_t ridge_key(int32_t a, int32_t b, int32_t c) {
  uint64_t x = (uint64_t)(a + 1), y = (uint64_t)(b + 1), z = (uint64_t)(c + 1);
  if (x > y) { uint64_t t = x; x = y; y = t; }
  if (y > z) { uint64_t t = y; y = z; z = t; }
  if (x > y) { uint64_t t = x; x = y; y = t; }
  return (x << (2 * kSiteBits)) | (y << kSiteBits) | z;
}

__device__ __forceinline__ uint64_t hash64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// --------------------------------------------------------------------------------------
// kernels
// --------------------------------------------------------------------------------------

// Decides every ridge pair: a new tetrahedron (flag 1, with its candidate count) or nothing.
__global__ void classify_kernel(const Item *__restrict__ items, int64_t w,
                                const int32_t *__restrict__ minc,
                                const int32_t *__restrict__ clen, uint32_t *__restrict__ isnew,
                                uint64_t *__restrict__ cand) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w) return;
  const Item it = items[i];
  const int32_t c1 = minc[it.t1], c2 = minc[it.t2];
  if (c1 == c2) {
    isnew[i] = 0;
    cand[i] = 0;
    return;
  }
  isnew[i] = 1;
  cand[i] = (uint64_t)clen[it.t1] + (uint64_t)clen[it.t2];
}

// Writes the new tetrahedron of every creating ridge pair (t1's vertices with its apex, the
// vertex not on the ridge, replaced by the creating site: the orientation is kept because
// that site lies on t1's side of the ridge) and its job; list entries (i, p) for the
// ridge's finite vertices.
__global__ void make_kernel(const Item *__restrict__ items, int64_t w,
                            const uint32_t *__restrict__ isnew,
                            const uint32_t *__restrict__ newpos,
                            const uint64_t *__restrict__ candoff, const int32_t *__restrict__ minc,
                            const int32_t *__restrict__ clen, int4 *__restrict__ tv,
                            int32_t *__restrict__ minc_out, Job *__restrict__ jobs,
                            uint64_t *__restrict__ jobstart, uint64_t *__restrict__ pairs,
                            int32_t tbase, uint32_t *__restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= w || !isnew[i]) return;
  Item it = items[i];
  int32_t td = it.t1, ts = it.t2;
  if (minc[ts] < minc[td]) { td = it.t2; ts = it.t1; }
  const int32_t p = minc[td];
  const int4 a = tv[td], b = tv[ts];
  int32_t va[4] = {a.x, a.y, a.z, a.w};
  const int32_t vb[4] = {b.x, b.y, b.z, b.w};
  int apex = -1, nshared = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool shared = va[k] == vb[0] || va[k] == vb[1] || va[k] == vb[2] || va[k] == vb[3];
    if (!shared) apex = k;
    nshared += shared ? 1 : 0;
  }
  if (nshared != 3) {
    atomicOr(err, kErrRidge);
    apex = 0;   // keeps every index in range; the host stops after this round
  }
  const int32_t tnew = tbase + (int32_t)newpos[i];
  uint64_t *pr = pairs + 3 * (int64_t)tnew;
  int m = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k == apex) continue;
    pr[m++] = va[k] < 0 ? ~0ull : (((uint64_t)(uint32_t)va[k] << 32) | (uint32_t)p);
  }
  va[apex] = p;
  tv[tnew] = make_int4(va[0], va[1], va[2], va[3]);
  minc_out[tnew] = kNone;
  Job j;
  j.tnew = tnew;
  j.td = td;
  j.ts = ts;
  j.p = p;
  j.nd = clen[td];
  j.apex = apex;
  jobs[newpos[i]] = j;
  jobstart[newpos[i]] = candoff[i];
}

// One thread per candidate test: finds its job (the last job starting at or before it),
// takes the candidate from td's list, then ts's, and writes 1 (in the new conflict list),
// 0, or 2 (deferred to the host).  A candidate at the creating site's own coordinates is a
// duplicate point.  The accepted candidates' smallest site per job is reduced in LDS (a
// block spans at most 256 jobs) and then joins the job's min conflict with one atomic.
__global__ __launch_bounds__(256) void test_kernel(
    const Job *__restrict__ jobs, const uint64_t *__restrict__ jobstart, int64_t njobs,
    uint64_t c0, uint64_t ncand, const int4 *__restrict__ tv, const int64_t *__restrict__ coff,
    const int32_t *__restrict__ pool, const float4 *__restrict__ P, uint8_t *__restrict__ flag,
    int32_t *__restrict__ candq, int32_t *__restrict__ minc, Deferred *__restrict__ deferred,
    uint32_t *__restrict__ ndeferred, uint32_t max_deferred, int32_t *__restrict__ dup) {
  const uint64_t idx = c0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // the jobs this block covers: [s_lo, s_hi], found once by the first lane
  __shared__ int64_t s_lo, s_hi;
  __shared__ int32_t s_min[256];
  s_min[threadIdx.x] = kNone;
  if (threadIdx.x == 0) {
    const uint64_t first = c0 + (uint64_t)blockIdx.x * blockDim.x;
    const uint64_t last = min(first + blockDim.x, ncand) - 1;
    int64_t lo = 0, hi = njobs - 1;
    while (lo < hi) {   // last job with start <= first
      const int64_t mid = (lo + hi + 1) >> 1;
      if (jobstart[mid] <= first) lo = mid; else hi = mid - 1;
    }
    int64_t lo2 = lo, hi2 = njobs - 1;
    while (lo2 < hi2) {  // last job with start <= last
      const int64_t mid = (lo2 + hi2 + 1) >> 1;
      if (jobstart[mid] <= last) lo2 = mid; else hi2 = mid - 1;
    }
    s_lo = lo;
    s_hi = lo2;
  }
  __syncthreads();
  if (idx < ncand) {
    int64_t lo = s_lo, hi = s_hi;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (jobstart[mid] <= idx) lo = mid; else hi = mid - 1;
    }
    const Job j = jobs[lo];
    const int64_t e = (int64_t)(idx - jobstart[lo]);
    const bool from_td = e < j.nd;
    const int32_t q = from_td ? pool[coff[j.td] + e] : pool[coff[j.ts] + (e - j.nd)];
    candq[idx] = q;
    int c = 0;
    if (q != j.p) {
      const double3 xq = site(P, q);
      c = conflict_filter(P, tv[j.tnew], xq);
      if (c == 1 && !from_td) {
        const int c2 = conflict_filter(P, tv[j.td], xq);   // already in td's list?
        c = c2 == 0 ? 1 : (c2 == 1 ? 0 : 2);
      }
      if (c == 2) {
        if (j.p >= 0) {
          const float4 a = P[q], b = P[j.p];
          if (a.x == b.x && a.y == b.y && a.z == b.z) atomicMin(dup, q);
        }
        const uint32_t s = atomicAdd(ndeferred, 1u);
        if (s < max_deferred) {
          Deferred d;
          const int4 v = tv[j.tnew], vd = tv[j.td];
          d.v[0] = v.x; d.v[1] = v.y; d.v[2] = v.z; d.v[3] = v.w;
          d.vd[0] = vd.x; d.vd[1] = vd.y; d.vd[2] = vd.z; d.vd[3] = vd.w;
          d.q = q;
          d.from_td = from_td ? 1 : 0;
          d.idx = (int64_t)idx;
          d.tnew = j.tnew;
          d.pad = 0;
          deferred[s] = d;
        }
      }
      if (c == 1) atomicMin(&s_min[lo - s_lo], q);
    }
    flag[idx] = (uint8_t)c;
  }
  __syncthreads();
  const int64_t nj = s_hi - s_lo + 1;
  if ((int64_t)threadIdx.x < nj && s_min[threadIdx.x] != kNone)
    atomicMin(&minc[jobs[s_lo + threadIdx.x].tnew], s_min[threadIdx.x]);
}

// Deferred signs decided on the host: the verdict goes to the flag, and an accepted
// candidate joins its tetrahedron's min conflict.
__global__ void settle_kernel(const Deferred *__restrict__ deferred,
                              const uint8_t *__restrict__ verdict, uint32_t n,
                              uint8_t *__restrict__ flag, int32_t *__restrict__ minc) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Deferred d = deferred[i];
  flag[d.idx] = verdict[i];
  if (verdict[i]) atomicMin(&minc[d.tnew], d.q);
}

// Accepted candidates go to their packed place in the pool.
__global__ void write_kernel(const uint8_t *__restrict__ flag, const uint64_t *__restrict__ pos,
                             const int32_t *__restrict__ candq, uint64_t ncand,
                             int64_t pool_base, int32_t *__restrict__ pool) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < ncand && flag[idx]) pool[pool_base + (int64_t)pos[idx]] = candq[idx];
}

// Each job's packed list range; then its ridge pairs for the next round: (tnew, ts) on the
// ridge it was created on, and through the hash table the pairs of its three ridges
// through the creating site.
__global__ void finish_kernel(const Job *__restrict__ jobs, const uint64_t *__restrict__ jobstart,
                              int64_t njobs, const uint64_t *__restrict__ pos, uint64_t ncand,
                              uint64_t naccepted, int64_t pool_base, const int4 *__restrict__ tv,
                              int64_t *__restrict__ coff, int32_t *__restrict__ clen,
                              uint64_t *__restrict__ hkey, int32_t *__restrict__ hval,
                              uint64_t hmask, Item *__restrict__ next,
                              uint32_t *__restrict__ nnext, int checkin,
                              uint32_t *__restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= njobs) return;
  const Job j = jobs[i];
  const uint64_t s = jobstart[i];
  const uint64_t e = (i + 1 < njobs) ? jobstart[i + 1] : ncand;
  const uint64_t ps = s < ncand ? pos[s] : naccepted;
  const uint64_t pe = e < ncand ? pos[e] : naccepted;
  coff[j.tnew] = pool_base + (int64_t)ps;
  clen[j.tnew] = (int32_t)(pe - ps);
  if (!checkin) return;
  uint32_t o = atomicAdd(nnext, 1u);
  next[o] = Item{j.tnew, j.ts};
  const int4 t = tv[j.tnew];
  const int32_t v[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k == j.apex) continue;
    int32_t f[3];
    int m = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l)
      if (l != k) f[m++] = v[l];
    const uint64_t key = ridge_key(f[0], f[1], f[2]);
    uint64_t h = hash64(key) & hmask;
    int probes = 0;
    for (;;) {
      const uint64_t old = atomicCAS((unsigned long long *)&hkey[h], (unsigned long long)kEmptyKey,
                                     (unsigned long long)key);
      if (old == kEmptyKey || old == key) break;
      h = (h + 1) & hmask;
      if (++probes == kMaxProbes) break;
    }
    if (probes == kMaxProbes) {
      atomicOr(err, kErrTable);
      continue;
    }
    const int32_t other = atomicExch(&hval[h], j.tnew);
    if (other != kEmptyVal) {
      o = atomicAdd(nnext, 1u);
      next[o] = Item{j.tnew, other};
    }
  }
}

// Low-dimensional start: entries by position become entries by rank; an entry stays only
// when its owner is an older real rank than its successor (a rank on the start's line or
// plane has, among the older ranks, exactly its neighbours in the prefix's diagram, and the
// start's later ranks and spare points own nothing here).
__global__ void rank_pairs_kernel(uint64_t *pairs, int64_t m, const int32_t *rank_of_pos,
                                  int64_t nreal) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m || pairs[e] == ~0ull) return;
  const int64_t i = rank_of_pos[pairs[e] >> 32], j = rank_of_pos[(uint32_t)pairs[e]];
  pairs[e] = (i < j && j < nreal) ? (((uint64_t)i << 32) | (uint64_t)j) : ~0ull;
}

// Entries (i, x) for every rank i < x: the start's ranks A and B (the first off the line,
// the first off the plane) join every older list.
__global__ void older_pairs_kernel(uint64_t *out, int64_t x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < x) out[i] = ((uint64_t)i << 32) | (uint64_t)x;
}

__global__ void fill_u64_kernel(uint64_t *p, uint64_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void iota_kernel(int32_t *p, int32_t from, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = from + (int32_t)i;
}

// Re-inserts the ridges still waiting for their second tetrahedron into a larger table.
__global__ void rehash_kernel(const uint64_t *__restrict__ okey, const int32_t *__restrict__ oval,
                              uint64_t osize, uint64_t *__restrict__ hkey,
                              int32_t *__restrict__ hval, uint64_t hmask,
                              uint32_t *__restrict__ err) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= osize || okey[i] == kEmptyKey) return;
  uint64_t h = hash64(okey[i]) & hmask;
  for (int probes = 0;; ++probes) {
    if (probes == kMaxProbes) {
      atomicOr(err, kErrTable);
      return;
    }
    const uint64_t old = atomicCAS((unsigned long long *)&hkey[h], (unsigned long long)kEmptyKey,
                                   (unsigned long long)okey[i]);
    if (old == kEmptyKey) break;
    h = (h + 1) & hmask;
  }
  hval[h] = oval[i];
}

// Sorted unique entries (owner << 32 | successor) to CSR: ranks and the first entry of
// every owner.
__global__ void csr_kernel(const uint64_t *__restrict__ key, int64_t nnz, int64_t n,
                           int32_t *__restrict__ ent, int64_t *__restrict__ off) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e > nnz) return;
  const int64_t own = e < nnz ? (int64_t)(key[e] >> 32) : n;
  const int64_t prev = e > 0 ? (int64_t)(key[e - 1] >> 32) : -1;
  for (int64_t r = prev + 1; r <= own; ++r) off[r] = e;
  if (e < nnz) ent[e] = (int32_t)(uint32_t)key[e];
}

__global__ void swap_kernel(const uint64_t *__restrict__ in, int64_t m, uint64_t *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) out[e] = (in[e] << 32) | (in[e] >> 32);
}

__global__ void unique_flag_kernel(const uint64_t *__restrict__ key, int64_t m,
                                   uint32_t *__restrict__ keep) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  keep[e] = (key[e] != ~0ull) && (e == 0 || key[e] != key[e - 1]);
}

__global__ void compact_kernel(const uint64_t *__restrict__ key, const uint32_t *__restrict__ keep,
                               const uint32_t *__restrict__ pos, int64_t m,
                               uint64_t *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m && keep[e]) out[pos[e]] = key[e];
}

// --------------------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------------------

// The construction's conflict test, exactly (host predicates): q newer than every vertex.
static bool conflict_exact(const std::vector<double> &P, const int32_t v[4], const double *q) {
  auto pt = [&](int32_t i) { return &P[3 * (size_t)i]; };
  int inf = -1;
  for (int i = 0; i < 4; ++i)
    if (v[i] < 0) inf = i;
  if (inf < 0) return insphere(pt(v[0]), pt(v[1]), pt(v[2]), pt(v[3]), q) >= 0;
  const double *x[4];
  for (int i = 0; i < 4; ++i) x[i] = (i == inf) ? q : pt(v[i]);
  const int o = orient3d(x[0], x[1], x[2], x[3]);
  if (o != 0) return o > 0;
  // q in the facet's plane: its circumcircle, through an auxiliary point beyond the facet
  const double *a = pt(v[(inf + 1) & 3]);
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 2; ++s) {
      double f[3] = {a[0], a[1], a[2]};
      f[k] = s == 0 ? a[k] + 1.0 : a[k] - 1.0;
      const double *r[4];
      for (int i = 0; i < 4; ++i) r[i] = (i == inf) ? f : pt(v[i]);
      if (orient3d(r[0], r[1], r[2], r[3]) > 0) return insphere(r[0], r[1], r[2], r[3], q) >= 0;
    }
  return false;
}

#define GB_CHECK(x)                                                                        \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) throw std::runtime_error(std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
struct DevBuf {
  T *p = nullptr;
  int64_t cap = 0;
  ~DevBuf() { if (p) (void)hipFree(p); }
  void reserve(int64_t n, hipStream_t st, bool keep = false, int64_t used = 0) {
    if (n <= cap) return;
    int64_t c = std::max<int64_t>(n, cap + cap / 2);
    T *q = nullptr;
    GB_CHECK(hipMalloc(&q, sizeof(T) * (size_t)c));
    if (keep && p && used > 0)
      GB_CHECK(hipMemcpyAsync(q, p, sizeof(T) * (size_t)used, hipMemcpyDeviceToDevice, st));
    if (p) {
      GB_CHECK(hipStreamSynchronize(st));
      GB_CHECK(hipFree(p));
    }
    p = q;
    cap = c;
  }
};

struct ByteToU64 {
  __host__ __device__ uint64_t operator()(uint8_t v) const { return v; }
};

static inline unsigned blocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

struct Stats {
  int64_t rounds = 0, tets = 0, conflicts = 0, tests = 0, deferred = 0, entries = 0;
  double ms = 0;
};

// A start from ranks 0, 1, A, B when the first four ranks are coplanar (the host
// construction's low-dimensional plan): the sites are then inserted in the order 0, 1, A,
// B, the other real ranks ascending; A or B may be a spare point off the line or plane.
struct LowDim {
  std::vector<int32_t> rank_of_pos;   // rank (spares: nreal, nreal + 1) of each position
  int64_t nreal = 0;
  int32_t A = -1, B = -1;
};

// Successor lists of the sites at positions 0..n-1 of P (the insertion order).  Without a
// low-dimensional plan the positions are the ranks: list i holds the later positions j
// whose insertion created tetrahedra with i on the cavity boundary, plus the start's pairs.
// With one, the entries are mapped to ranks as the host construction records them.
// Throws the position of a duplicate site (int64_t), or std::runtime_error.
static int64_t build_positions(const std::vector<double> &P, int64_t n, hipStream_t st, Csr *succ,
                               Csr *pred, Stats *stats, const LowDim *ld = nullptr) {
  auto t0 = std::chrono::steady_clock::now();
  // sites as float4 (the inputs are float32; the host predicates see the same values)
  std::vector<float> P4(4 * (size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) P4[4 * i + k] = (float)P[3 * i + k];
    P4[4 * i + 3] = 0.f;
  }
  DevBuf<float4> dP;
  dP.reserve(n, st);
  GB_CHECK(hipMemcpyAsync(dP.p, P4.data(), sizeof(float4) * (size_t)n, hipMemcpyHostToDevice, st));

  // tetrahedra
  // capacities from measured ratios (tetrahedra created: 18-25 per point on surfaces, up to
  // 29 on lattices; conflict records: about 800 per point for 1M surface points), grown
  // when exceeded
  int64_t tcap = 30 * n + 4096;
  DevBuf<int4> tv;
  DevBuf<int32_t> minc, clen;
  DevBuf<int64_t> coff;
  DevBuf<uint64_t> pairs;
  tv.reserve(tcap, st);
  minc.reserve(tcap, st);
  clen.reserve(tcap, st);
  coff.reserve(tcap, st);
  pairs.reserve(3 * tcap, st);
  int64_t ntet = 0;
  // conflict pool
  DevBuf<int32_t> pool;
  pool.reserve(256 * n + 4096, st);
  int64_t pool_used = 0;
  // ridge hash table (faces checked in so far); load factor below one half
  uint64_t hsize = 1;
  while (hsize < (uint64_t)(3 * tcap)) hsize <<= 1;
  DevBuf<uint64_t> hkey;
  DevBuf<int32_t> hval;
  hkey.reserve((int64_t)hsize, st);
  hval.reserve((int64_t)hsize, st);
  fill_u64_kernel<<<blocks(hsize), 256, 0, st>>>(hkey.p, kEmptyKey, (int64_t)hsize);
  fill_i32_kernel<<<blocks(hsize), 256, 0, st>>>(hval.p, kEmptyVal, (int64_t)hsize);

  // per-round buffers
  DevBuf<Item> items, next;
  DevBuf<uint32_t> isnew, newpos, nnext;
  DevBuf<uint64_t> cand, candoff, jobstart, pos;
  DevBuf<Job> jobs;
  DevBuf<uint8_t> flag, verdict;
  DevBuf<int32_t> candq, dup;
  DevBuf<Deferred> deferred;
  DevBuf<uint32_t> ndeferred, err;
  DevBuf<uint8_t> scratch;
  err.reserve(1, st);
  GB_CHECK(hipMemsetAsync(err.p, 0, sizeof(uint32_t), st));
  auto check_err = [&]() {
    uint32_t e = 0;
    GB_CHECK(hipMemcpyAsync(&e, err.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GB_CHECK(hipStreamSynchronize(st));
    if (e & kErrRidge) throw std::runtime_error("internal: a ridge pair without a common triangle");
    if (e & kErrTable) throw std::runtime_error("internal: ridge table full");
  };
  nnext.reserve(1, st);
  ndeferred.reserve(1, st);
  dup.reserve(1, st);
  const uint32_t max_deferred = 1u << 20;
  deferred.reserve(max_deferred, st);
  verdict.reserve(max_deferred, st);
  fill_i32_kernel<<<1, 1, 0, st>>>(dup.p, INT32_MAX, 1);
  auto scan_u32 = [&](const uint32_t *in, uint32_t *out, int64_t m) {
    size_t bytes = 0;
    GB_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)m, st));
    scratch.reserve((int64_t)bytes + 16, st);
    GB_CHECK(hipcub::DeviceScan::ExclusiveSum(scratch.p, bytes, in, out, (int)m, st));
  };
  auto scan_u64 = [&](const uint64_t *in, uint64_t *out, int64_t m) {
    size_t bytes = 0;
    GB_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)m, st));
    scratch.reserve((int64_t)bytes + 16, st);
    GB_CHECK(hipcub::DeviceScan::ExclusiveSum(scratch.p, bytes, in, out, (int)m, st));
  };
  std::vector<Deferred> hdef;
  std::vector<uint8_t> hver;

  // Tests the candidates of njobs jobs (their Job records and start offsets already on the
  // device), settles deferred ones on the host, packs the accepted ones into the pool and
  // sets each new tetrahedron's list; with checkin, emits the next round's ridge pairs.
  // Returns the number of pairs emitted.
  flag.reserve(8 * n + 4096, st);
  candq.reserve(8 * n + 4096, st);
  pos.reserve(8 * n + 4096, st);
  auto run_jobs = [&](int64_t njobs, uint64_t ncand, bool checkin) -> uint32_t {
    flag.reserve((int64_t)ncand + 1, st);
    candq.reserve((int64_t)ncand + 1, st);
    pos.reserve((int64_t)ncand + 1, st);
    // test in slices; a slice whose deferred signs overflow the buffer is tested again in
    // halves (the test writes only its own candidates' flags, so repeating it is harmless)
    uint64_t slice = ncand;
    for (uint64_t c0 = 0; c0 < ncand;) {
      const uint64_t len = std::min(slice, ncand - c0);
      GB_CHECK(hipMemsetAsync(ndeferred.p, 0, sizeof(uint32_t), st));
      test_kernel<<<blocks((int64_t)len), 256, 0, st>>>(
          jobs.p, jobstart.p, njobs, c0, c0 + len, tv.p, coff.p, pool.p, dP.p, flag.p, candq.p,
          minc.p, deferred.p, ndeferred.p, max_deferred, dup.p);
      uint32_t nd = 0;
      int32_t hdup = 0;
      GB_CHECK(hipMemcpyAsync(&nd, ndeferred.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
      GB_CHECK(hipMemcpyAsync(&hdup, dup.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      GB_CHECK(hipStreamSynchronize(st));
      if (hdup != INT32_MAX) throw (int64_t)hdup;
      if (nd > max_deferred) {
        if (len == 1) throw std::runtime_error("internal: deferred buffer");
        slice = std::max<uint64_t>(1, len / 2);
        continue;
      }
      stats->deferred += nd;
      if (nd > 0) {
        hdef.resize(nd);
        hver.resize(nd);
        GB_CHECK(hipMemcpyAsync(hdef.data(), deferred.p, sizeof(Deferred) * nd,
                                hipMemcpyDeviceToHost, st));
        GB_CHECK(hipStreamSynchronize(st));
        for (uint32_t i = 0; i < nd; ++i) {
          const Deferred &d = hdef[i];
          const double *q = &P[3 * (size_t)d.q];
          bool c = conflict_exact(P, d.v, q);
          if (c && !d.from_td) c = !conflict_exact(P, d.vd, q);
          hver[i] = c ? 1 : 0;
        }
        GB_CHECK(hipMemcpyAsync(verdict.p, hver.data(), nd, hipMemcpyHostToDevice, st));
        settle_kernel<<<blocks(nd), 256, 0, st>>>(deferred.p, verdict.p, nd, flag.p, minc.p);
      }
      c0 += len;
    }
    stats->tests += (int64_t)ncand;
    // packed positions of the accepted candidates
    uint64_t nacc = 0;
    if (ncand > 0) {
      // the sum runs in the input's type: read the byte flags as 64-bit counts
      hipcub::TransformInputIterator<uint64_t, ByteToU64, const uint8_t *> fl(flag.p, ByteToU64());
      size_t bytes = 0;
      GB_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, fl, pos.p, (int64_t)ncand, st));
      scratch.reserve((int64_t)bytes + 16, st);
      GB_CHECK(hipcub::DeviceScan::ExclusiveSum(scratch.p, bytes, fl, pos.p, (int64_t)ncand, st));
      uint64_t lastpos = 0;
      uint8_t lastflag = 0;
      GB_CHECK(hipMemcpyAsync(&lastpos, pos.p + ncand - 1, 8, hipMemcpyDeviceToHost, st));
      GB_CHECK(hipMemcpyAsync(&lastflag, flag.p + ncand - 1, 1, hipMemcpyDeviceToHost, st));
      GB_CHECK(hipStreamSynchronize(st));
      nacc = lastpos + lastflag;
    }
    pool.reserve(pool_used + (int64_t)nacc + 1, st, true, pool_used);
    if (ncand > 0)
      write_kernel<<<blocks((int64_t)ncand), 256, 0, st>>>(flag.p, pos.p, candq.p, ncand,
                                                           pool_used, pool.p);
    GB_CHECK(hipMemsetAsync(nnext.p, 0, sizeof(uint32_t), st));
    finish_kernel<<<blocks(njobs), 256, 0, st>>>(jobs.p, jobstart.p, njobs, pos.p, ncand, nacc,
                                                 pool_used, tv.p, coff.p, clen.p, hkey.p, hval.p,
                                                 hsize - 1, next.p, nnext.p, checkin ? 1 : 0,
                                                 err.p);
    pool_used += (int64_t)nacc;
    stats->conflicts += (int64_t)nacc;
    uint32_t nn = 0;
    GB_CHECK(hipMemcpyAsync(&nn, nnext.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GB_CHECK(hipStreamSynchronize(st));
    return nn;
  };

  // --- start: the first tetrahedron and its four ghosts (as the sequential construction
  // sets them up), filled from a universe tetrahedron whose list is every later site
  {
    auto pt = [&](int32_t i) { return &P[3 * (size_t)i]; };
    int32_t v[4] = {0, 1, 2, 3};
    const int o = orient3d(pt(0), pt(1), pt(2), pt(3));
    if (o == 0) throw std::runtime_error("degenerate start");
    if (o < 0) std::swap(v[2], v[3]);
    std::vector<int4> t0(6);
    t0[0] = make_int4(v[0], v[1], v[2], v[3]);
    for (int i = 0; i < 4; ++i) {
      int32_t w[4] = {v[0], v[1], v[2], v[3]};
      w[i] = -1;
      std::swap(w[(i + 1) & 3], w[(i + 2) & 3]);
      t0[1 + i] = make_int4(w[0], w[1], w[2], w[3]);
    }
    t0[5] = make_int4(-1, -1, -1, -1);   // the universe: never a tetrahedron of the result
    GB_CHECK(hipMemcpyAsync(tv.p, t0.data(), sizeof(int4) * 6, hipMemcpyHostToDevice, st));
    ntet = 6;
    fill_i32_kernel<<<1, 64, 0, st>>>(minc.p, kNone, 6);
    iota_kernel<<<blocks(n - 4), 256, 0, st>>>(pool.p, 4, n - 4);
    pool_used = n - 4;
    const int64_t c5 = 0;
    const int32_t l5 = (int32_t)(n - 4);
    GB_CHECK(hipMemcpyAsync(coff.p + 5, &c5, 8, hipMemcpyHostToDevice, st));
    GB_CHECK(hipMemcpyAsync(clen.p + 5, &l5, 4, hipMemcpyHostToDevice, st));
    std::vector<Job> j0(5);
    std::vector<uint64_t> s0(5);
    for (int i = 0; i < 5; ++i) {
      j0[i] = Job{i, 5, -1, -1, l5, -1};
      s0[i] = (uint64_t)i * (uint64_t)l5;
    }
    jobs.reserve(5, st);
    jobstart.reserve(5, st);
    next.reserve(16, st);
    GB_CHECK(hipMemcpyAsync(jobs.p, j0.data(), sizeof(Job) * 5, hipMemcpyHostToDevice, st));
    GB_CHECK(hipMemcpyAsync(jobstart.p, s0.data(), sizeof(uint64_t) * 5, hipMemcpyHostToDevice, st));
    run_jobs(5, 5 * (uint64_t)l5, false);
    // the start's list entries: every pair of the first four sites (low-dimensional start:
    // only ranks 0 and 1, whose bisector plane is their common facet)
    std::vector<uint64_t> e0;
    for (int j = 1; j < 4; ++j)
      for (int i = 0; i < j; ++i)
        if (!ld || j == 1) e0.push_back(((uint64_t)i << 32) | (uint64_t)j);
    while (e0.size() < 18) e0.push_back(~0ull);   // pair slots of the six start tetrahedra
    GB_CHECK(hipMemcpyAsync(pairs.p, e0.data(), sizeof(uint64_t) * 18, hipMemcpyHostToDevice, st));
    // the ten ridge pairs of the start
    std::vector<Item> w0;
    for (int a = 0; a < 5; ++a)
      for (int b = a + 1; b < 5; ++b) w0.push_back(Item{a, b});
    items.reserve(16, st);
    GB_CHECK(hipMemcpyAsync(items.p, w0.data(), sizeof(Item) * w0.size(), hipMemcpyHostToDevice, st));
    GB_CHECK(hipStreamSynchronize(st));   // the host vectors above end with this block
  }
  int64_t w = 10;
  while (w > 0) {
    ++stats->rounds;
    isnew.reserve(w + 1, st);
    newpos.reserve(w + 1, st);
    cand.reserve(w + 1, st);
    candoff.reserve(w + 1, st);
    classify_kernel<<<blocks(w), 256, 0, st>>>(items.p, w, minc.p, clen.p, isnew.p, cand.p);
    scan_u32(isnew.p, newpos.p, w);
    scan_u64(cand.p, candoff.p, w);
    uint32_t lastnew = 0, lastflag = 0;
    uint64_t lastoff = 0, lastcand = 0;
    GB_CHECK(hipMemcpyAsync(&lastnew, newpos.p + w - 1, 4, hipMemcpyDeviceToHost, st));
    GB_CHECK(hipMemcpyAsync(&lastflag, isnew.p + w - 1, 4, hipMemcpyDeviceToHost, st));
    GB_CHECK(hipMemcpyAsync(&lastoff, candoff.p + w - 1, 8, hipMemcpyDeviceToHost, st));
    GB_CHECK(hipMemcpyAsync(&lastcand, cand.p + w - 1, 8, hipMemcpyDeviceToHost, st));
    GB_CHECK(hipStreamSynchronize(st));
    const int64_t njobs = (int64_t)lastnew + lastflag;
    const uint64_t ncand = lastoff + lastcand;
    if (njobs == 0) break;
    if (ntet + njobs > tcap) {   // more tetrahedra: grow the arrays and the ridge table
      const int64_t nc = std::max<int64_t>(ntet + njobs, tcap + tcap / 2);
      tv.reserve(nc, st, true, ntet);
      minc.reserve(nc, st, true, ntet);
      clen.reserve(nc, st, true, ntet);
      coff.reserve(nc, st, true, ntet);
      pairs.reserve(3 * nc, st, true, 3 * ntet);
      tcap = nc;
      uint64_t hs = hsize;
      while (hs < (uint64_t)(3 * tcap)) hs <<= 1;
      if (hs != hsize) {
        DevBuf<uint64_t> k2;
        DevBuf<int32_t> v2;
        k2.reserve((int64_t)hs, st);
        v2.reserve((int64_t)hs, st);
        fill_u64_kernel<<<blocks(hs), 256, 0, st>>>(k2.p, kEmptyKey, (int64_t)hs);
        fill_i32_kernel<<<blocks(hs), 256, 0, st>>>(v2.p, kEmptyVal, (int64_t)hs);
        rehash_kernel<<<blocks(hsize), 256, 0, st>>>(hkey.p, hval.p, hsize, k2.p, v2.p, hs - 1,
                                                     err.p);
        GB_CHECK(hipStreamSynchronize(st));
        std::swap(hkey.p, k2.p);
        std::swap(hkey.cap, k2.cap);
        std::swap(hval.p, v2.p);
        std::swap(hval.cap, v2.cap);
        hsize = hs;
      }
    }
    jobs.reserve(njobs + 1, st);
    jobstart.reserve(njobs + 1, st);
    make_kernel<<<blocks(w), 256, 0, st>>>(items.p, w, isnew.p, newpos.p, candoff.p, minc.p,
                                           clen.p, tv.p, minc.p, jobs.p, jobstart.p, pairs.p,
                                           (int32_t)ntet, err.p);
    ntet += njobs;
    next.reserve(4 * njobs + 1, st);
    const uint32_t nn = run_jobs(njobs, ncand, true);
    check_err();
    std::swap(items.p, next.p);
    std::swap(items.cap, next.cap);
    w = nn;
  }
  stats->tets = ntet - 1;   // the universe is no tetrahedron

  // entries (owner << 32 | successor): sort, drop repeats and the ghost slots, to CSR
  int64_t m = 3 * ntet;
  int64_t nout = n;   // lists produced
  if (ld) {
    DevBuf<int32_t> rop;
    rop.reserve(n, st);
    GB_CHECK(hipMemcpyAsync(rop.p, ld->rank_of_pos.data(), sizeof(int32_t) * n,
                            hipMemcpyHostToDevice, st));
    rank_pairs_kernel<<<blocks(m), 256, 0, st>>>(pairs.p, m, rop.p, ld->nreal);
    const int64_t xa = ld->A < ld->nreal ? ld->A : 0, xb = ld->B < ld->nreal ? ld->B : 0;
    pairs.reserve(m + xa + xb + 1, st, true, m);
    if (xa > 0) older_pairs_kernel<<<blocks(xa), 256, 0, st>>>(pairs.p + m, xa);
    if (xb > 0) older_pairs_kernel<<<blocks(xb), 256, 0, st>>>(pairs.p + m + xa, xb);
    m += xa + xb;
    nout = ld->nreal;
    GB_CHECK(hipStreamSynchronize(st));   // rop ends with this block
  }
  DevBuf<uint64_t> sorted, uniq;
  DevBuf<uint32_t> keep, kpos;
  sorted.reserve(m, st);
  {
    size_t bytes = 0;
    GB_CHECK(hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, pairs.p, sorted.p, (int)m, 0, 64, st));
    scratch.reserve((int64_t)bytes + 16, st);
    GB_CHECK(hipcub::DeviceRadixSort::SortKeys(scratch.p, bytes, pairs.p, sorted.p, (int)m, 0, 64, st));
  }
  keep.reserve(m, st);
  kpos.reserve(m, st);
  unique_flag_kernel<<<blocks(m), 256, 0, st>>>(sorted.p, m, keep.p);
  scan_u32(keep.p, kpos.p, m);
  uint32_t lk = 0, lp = 0;
  GB_CHECK(hipMemcpyAsync(&lk, keep.p + m - 1, 4, hipMemcpyDeviceToHost, st));
  GB_CHECK(hipMemcpyAsync(&lp, kpos.p + m - 1, 4, hipMemcpyDeviceToHost, st));
  GB_CHECK(hipStreamSynchronize(st));
  const int64_t nnz = (int64_t)lk + lp;
  uniq.reserve(nnz + 1, st);
  compact_kernel<<<blocks(m), 256, 0, st>>>(sorted.p, keep.p, kpos.p, m, uniq.p);
  DevBuf<int32_t> ent;
  DevBuf<int64_t> off;
  ent.reserve(nnz + 1, st);
  off.reserve(nout + 1, st);
  csr_kernel<<<blocks(nnz + 1), 256, 0, st>>>(uniq.p, nnz, nout, ent.p, off.p);
  succ->off.resize(nout + 1);
  succ->ent.resize(nnz);
  GB_CHECK(hipMemcpyAsync(succ->off.data(), off.p, sizeof(int64_t) * (nout + 1),
                          hipMemcpyDeviceToHost, st));
  if (nnz > 0)
    GB_CHECK(hipMemcpyAsync(succ->ent.data(), ent.p, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
  // (the copies above are ordered before the transpose below reuses ent and off on `st`)
  // predecessors (the transpose): the same entries keyed (successor << 32 | owner), sorted
  if (pred) {
    swap_kernel<<<blocks(nnz), 256, 0, st>>>(uniq.p, nnz, sorted.p);
    size_t bytes = 0;
    GB_CHECK(hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, sorted.p, uniq.p, (int)nnz, 0, 64, st));
    scratch.reserve((int64_t)bytes + 16, st);
    GB_CHECK(hipcub::DeviceRadixSort::SortKeys(scratch.p, bytes, sorted.p, uniq.p, (int)nnz, 0, 64, st));
    csr_kernel<<<blocks(nnz + 1), 256, 0, st>>>(uniq.p, nnz, nout, ent.p, off.p);
    pred->off.resize(nout + 1);
    pred->ent.resize(nnz);
    GB_CHECK(hipMemcpyAsync(pred->off.data(), off.p, sizeof(int64_t) * (nout + 1),
                            hipMemcpyDeviceToHost, st));
    if (nnz > 0)
      GB_CHECK(hipMemcpyAsync(pred->ent.data(), ent.p, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
  }
  GB_CHECK(hipStreamSynchronize(st));
  stats->entries = nnz;
  stats->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return 0;
}

static thread_local Stats g_last;

// The first rank whose coordinates equal those of an older rank, or -1.
static int64_t first_duplicate(const std::vector<double> &P, int64_t n) {
  struct H {
    size_t operator()(const std::array<double, 3> &a) const {
      uint64_t h = 1469598103934665603ull;
      for (double v : a) {
        uint64_t b;
        std::memcpy(&b, &v, 8);
        h = (h ^ b) * 1099511628211ull;
      }
      return (size_t)h;
    }
  };
  std::unordered_set<std::array<double, 3>, H> seen;
  seen.reserve((size_t)n);
  for (int64_t r = 0; r < n; ++r)
    if (!seen.insert({P[3 * r], P[3 * r + 1], P[3 * r + 2]}).second) return r;
  return -1;
}

}  // namespace gbuild
}  // namespace mknn

using namespace mknn;

extern "C" {

mknn_status mknn_build_device(const float *xyz, int64_t n, const int32_t *order, void *stream,
                              mknn_cloud **out) {
  clear_error();
  gbuild::g_last = gbuild::Stats{};   // stays zero when the host construction takes the call
  if (!out) return set_error(MKNN_EINVAL, "mknn_build_device: out is NULL");
  *out = nullptr;
  if (!xyz) return set_error(MKNN_EINVAL, "mknn_build_device: xyz is NULL");
  if (n < 1) return set_error(MKNN_EINVAL, "mknn_build_device: n must be >= 1");
  if (n > gbuild::kMaxSites)
    return set_error(MKNN_EUNSUPPORTED, "mknn_build_device: n above 2^21 - 2");
  // small clouds and starts whose first four ranks are coplanar take the host construction
  // (same lists); so does everything the host construction rejects, with its own error
  std::vector<double> P;
  std::vector<int32_t> ord(n);
  if (order) {
    std::vector<char> seen(n, 0);
    for (int64_t r = 0; r < n; ++r) {
      const int32_t o = order[r];
      if (o < 0 || o >= n || seen[o])
        return set_error(MKNN_EINVAL, "mknn_build_device: order is not a permutation of 0..n-1");
      seen[o] = 1;
      ord[r] = o;
    }
  } else {
    for (int64_t r = 0; r < n; ++r) ord[r] = (int32_t)r;
  }
  try {
    P.resize(3 * (size_t)n);
    for (int64_t r = 0; r < n; ++r)
      for (int k = 0; k < 3; ++k) {
        const float v = xyz[3 * (int64_t)ord[r] + k];
        if (!std::isfinite(v))
          return set_error(MKNN_ENONFINITE, "mknn_build_device: non-finite coordinate at point " +
                                                std::to_string(ord[r]));
        P[3 * r + k] = (double)v;
      }
  } catch (const std::bad_alloc &) {
    return set_error(MKNN_ENOMEM, "mknn_build_device: out of host memory");
  }
  if (n < 5) return mknn_build(xyz, n, order, out);
  // the first four ranks coplanar: the host construction's plan of a start off the line and
  // plane (A, B: ranks, or spare points appended after the real ones)
  gbuild::LowDim low;
  std::vector<double> Ppos;
  const bool lowdim = orient3d(&P[0], &P[3], &P[6], &P[9]) == 0;
  if (lowdim) {
    std::vector<double> P2(P);
    P2.resize(3 * (size_t)(n + 2));
    int64_t bad = -1;
    if (DelaunayBuilder::low_dim_plan(P2.data(), n, &low.A, &low.B, &bad) != kBuildOk)
      return mknn_build(xyz, n, order, out);   // (ranks 0 and 1 coincide: its error)
    low.nreal = n;
    low.rank_of_pos = {0, 1, low.A, low.B};
    for (int32_t r = 2; r < (int32_t)n; ++r)
      if (r != low.A && r != low.B) low.rank_of_pos.push_back(r);
    Ppos.resize(3 * low.rank_of_pos.size());
    for (size_t q = 0; q < low.rank_of_pos.size(); ++q)
      for (int k = 0; k < 3; ++k) Ppos[3 * q + k] = P2[3 * (size_t)low.rank_of_pos[q] + k];
  }
  const std::vector<double> &Pb = lowdim ? Ppos : P;
  const int64_t nb = (int64_t)(Pb.size() / 3);
  // a site at the coordinates of one of the four start sites would never be met as a
  // repeat of a creating site (the start sites create nothing): check those here
  for (int64_t r = 4; r < nb; ++r)
    for (int s = 0; s < 4; ++s)
      if (Pb[3 * r] == Pb[3 * s] && Pb[3 * r + 1] == Pb[3 * s + 1] &&
          Pb[3 * r + 2] == Pb[3 * s + 2]) {
        const int64_t first = gbuild::first_duplicate(P, n);
        return set_error(MKNN_EDUPLICATE, "mknn_build_device: point " +
                                              std::to_string(ord[first < 0 ? r : first]) +
                                              " duplicates an earlier point");
      }

  mknn_cloud *c = nullptr;
  try {
    gbuild::Stats st;
    Csr succ, pred;
    try {
      gbuild::build_positions(Pb, nb, (hipStream_t)stream, &succ, &pred, &st,
                              lowdim ? &low : nullptr);
    } catch (int64_t) {
      // a repeated site was met; name the first rank (in insertion order) that repeats an
      // older one, as the host construction does
      int64_t first = gbuild::first_duplicate(P, n);
      return set_error(MKNN_EDUPLICATE, "mknn_build_device: point " +
                                            std::to_string(ord[first < 0 ? 0 : first]) +
                                            " duplicates an earlier point");
    }
    gbuild::g_last = st;
    c = new mknn_cloud();
    c->n = n;
    c->order = ord;
    c->xyz.resize(3 * (size_t)n);
    for (int64_t i = 0; i < 3 * n; ++i) c->xyz[i] = (float)P[i];
    for (int k = 0; k < 3; ++k) {
      c->lo[k] = c->hi[k] = c->xyz[k];
      for (int64_t r = 1; r < n; ++r) {
        c->lo[k] = std::min(c->lo[k], c->xyz[3 * r + k]);
        c->hi[k] = std::max(c->hi[k], c->xyz[3 * r + k]);
      }
    }
    c->succ = std::move(succ);
    c->pred = std::move(pred);   // the transpose, sorted on the device
    c->live.assign(n, 1);
    c->nlive = n;
    c->head = 0;
  } catch (const std::bad_alloc &) {
    delete c;
    return set_error(MKNN_ENOMEM, "mknn_build_device: out of host memory");
  } catch (const std::exception &e) {
    delete c;
    return set_error(MKNN_EHIP, std::string("mknn_build_device: ") + e.what());
  }
  *out = c;
  return MKNN_OK;
}

mknn_status mknn_build_device_stats(int64_t counts[6], double *ms) {
  clear_error();
  if (!counts) return set_error(MKNN_EINVAL, "mknn_build_device_stats: counts is NULL");
  const gbuild::Stats &s = gbuild::g_last;
  counts[0] = s.rounds;
  counts[1] = s.tets;
  counts[2] = s.conflicts;
  counts[3] = s.tests;
  counts[4] = s.deferred;
  counts[5] = s.entries;
  if (ms) *ms = s.ms;
  return MKNN_OK;
}

}  // extern "C"
