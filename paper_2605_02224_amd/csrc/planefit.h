// Local plane fit on a finished k-NN row (the neighbourhood statistic the paper's scan
// convergence study computes from k = 20 nearest neighbours, Sec. 5.3.1): centroid c of the
// k' neighbours found, covariance C = (1/k') sum (p - c)(p - c)^T, normal = eigenvector of
// C's smallest eigenvalue lambda_0, residual sqrt(lambda_0) (the RMS distance of the
// neighbours to the plane) and surface variation lambda_0 / (lambda_0 + lambda_1 + lambda_2).
// The normal's largest-magnitude component is made positive (the first of equal ones).
// Fewer than three neighbours: normal, residual and variation are NaN (no neighbour at
// all: the centroid too).  All arithmetic in float64; output rounded to float32.
//
// One 16-lane row per query reads the query's k-NN row (slot 16 s + l in lane l) and loads
// its slots' points from the per-rank point array; the sums go through a 4-stage butterfly
// across the row, and every lane of the row then runs the same cyclic Jacobi iteration on
// the 3x3 matrix (all in registers, every index fixed at compile time).  A kernel of its
// own, launched on the query's stream right after the k-NN kernel: in the k-NN kernel's
// epilogue its registers would cost that kernel half its occupancy.
#pragma once
#include "knn_group.h"

namespace mknn {

constexpr int kPlaneFloats = 8;   // cx, cy, cz, nx, ny, nz, rms, variation

__device__ __forceinline__ double row_sum16(double v) {
  v += xor_lane_f64<1>(v);
  v += xor_lane_f64<2>(v);
  v += xor_lane_f64<4>(v);
  v += xor_lane_f64<8>(v);
  return v;
}

// One Jacobi rotation zeroing a[p][q] of the symmetric matrix held in (a00 .. a22), with
// the accumulated eigenvectors in the columns of v.  Written out per index pair so that
// nothing is addressed dynamically.
struct Sym3 {
  double a[3][3];
  double v[3][3];

  template <int P, int Q>
  __device__ __forceinline__ void rotate() {
    const double apq = a[P][Q];
    if (apq == 0.0) return;
    const double theta = (a[Q][Q] - a[P][P]) / (2.0 * apq);
    // the smaller root of t^2 + 2 t theta - 1 = 0, so the rotation angle is at most pi/4
    const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
    constexpr int R = 3 - P - Q;   // the third index
    const double arp = a[R][P], arq = a[R][Q];
    a[P][P] -= t * apq;
    a[Q][Q] += t * apq;
    a[P][Q] = a[Q][P] = 0.0;
    a[R][P] = a[P][R] = c * arp - s * arq;
    a[R][Q] = a[Q][R] = s * arp + c * arq;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double vip = v[i][P], viq = v[i][Q];
      v[i][P] = c * vip - s * viq;
      v[i][Q] = s * vip + c * viq;
    }
  }

  __device__ __forceinline__ void solve() {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) v[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 16; ++sweep) {
      const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
      const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
      if (!(off > 1e-36 * dia)) break;   // also ends on NaN
      rotate<0, 1>();
      rotate<0, 2>();
      rotate<1, 2>();
    }
  }
};

// Fit the plane of the row's neighbours and have lane 0 of the row write it.
template <int S>
__device__ __forceinline__ void row_plane_fit(const float4 *pts, const int32_t (&r)[S], int k,
                                              int l, float *out) {
  double px[S], py[S], pz[S];
  bool has[S];
  double sx = 0, sy = 0, sz = 0, cnt = 0;
#pragma unroll
  for (int t = 0; t < S; ++t) {
    has[t] = 16 * t + l < k && r[t] != kEmpty;
    px[t] = py[t] = pz[t] = 0.0;
    if (has[t]) {
      const float4 p = pts[r[t]];
      px[t] = p.x;
      py[t] = p.y;
      pz[t] = p.z;
      sx += px[t];
      sy += py[t];
      sz += pz[t];
      cnt += 1.0;
    }
  }
  sx = row_sum16(sx);
  sy = row_sum16(sy);
  sz = row_sum16(sz);
  cnt = row_sum16(cnt);
  const double cx = sx / cnt, cy = sy / cnt, cz = sz / cnt;
  double xx = 0, xy = 0, xz = 0, yy = 0, yz = 0, zz = 0;
#pragma unroll
  for (int t = 0; t < S; ++t) {
    if (has[t]) {
      const double dx = px[t] - cx, dy = py[t] - cy, dz = pz[t] - cz;
      xx += dx * dx;
      xy += dx * dy;
      xz += dx * dz;
      yy += dy * dy;
      yz += dy * dz;
      zz += dz * dz;
    }
  }
  Sym3 m;
  m.a[0][0] = row_sum16(xx) / cnt;
  m.a[0][1] = m.a[1][0] = row_sum16(xy) / cnt;
  m.a[0][2] = m.a[2][0] = row_sum16(xz) / cnt;
  m.a[1][1] = row_sum16(yy) / cnt;
  m.a[1][2] = m.a[2][1] = row_sum16(yz) / cnt;
  m.a[2][2] = row_sum16(zz) / cnt;
  m.solve();
  // the smallest eigenvalue (the first of equal ones) and its eigenvector
  const double l0 = m.a[0][0], l1 = m.a[1][1], l2 = m.a[2][2];
  const int i0 = (l0 <= l1 && l0 <= l2) ? 0 : (l1 <= l2 ? 1 : 2);
  double nx = i0 == 0 ? m.v[0][0] : (i0 == 1 ? m.v[0][1] : m.v[0][2]);
  double ny = i0 == 0 ? m.v[1][0] : (i0 == 1 ? m.v[1][1] : m.v[1][2]);
  double nz = i0 == 0 ? m.v[2][0] : (i0 == 1 ? m.v[2][1] : m.v[2][2]);
  const double lmin = fmax(i0 == 0 ? l0 : (i0 == 1 ? l1 : l2), 0.0);
  const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
  nx *= inv;
  ny *= inv;
  nz *= inv;
  const double ax = fabs(nx), ay = fabs(ny), az = fabs(nz);
  const double big = (ax >= ay && ax >= az) ? nx : (ay >= az ? ny : nz);
  if (big < 0.0) {
    nx = -nx;
    ny = -ny;
    nz = -nz;
  }
  const double tot = fmax(l0, 0.0) + fmax(l1, 0.0) + fmax(l2, 0.0);
  const bool fit = cnt >= 3.0;
  if (l == 0) {
    const float nan = __builtin_nanf("");
    out[0] = cnt > 0 ? (float)cx : nan;
    out[1] = cnt > 0 ? (float)cy : nan;
    out[2] = cnt > 0 ? (float)cz : nan;
    out[3] = fit ? (float)nx : nan;
    out[4] = fit ? (float)ny : nan;
    out[5] = fit ? (float)nz : nan;
    out[6] = fit ? (float)sqrt(lmin) : nan;
    out[7] = fit ? (float)(tot > 0.0 ? lmin / tot : 0.0) : nan;
  }
}

// One query per 16 lanes: idx is the k-NN output [nq][k] (rank, or -1 for padding).  With
// the Morton-sorted queries (qs, original index in w) the rows are taken in that order, so
// neighbouring rows gather neighbouring points.
template <int S>
__global__ __launch_bounds__(256) void plane_fit_kernel(const float4 *pts, const int32_t *idx,
                                                        const float4 *qs, int64_t nq, int k,
                                                        float *out) {
  const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int l = threadIdx.x & 15;
  if (s >= nq) return;   // whole rows leave together, so the row moves below stay in-row
  const int64_t q = qs ? (int64_t)__float_as_int(qs[s].w) : s;
  int32_t r[S];
#pragma unroll
  for (int t = 0; t < S; ++t) {
    const int j = 16 * t + l;
    const int32_t v = j < k ? idx[q * k + j] : -1;
    r[t] = v < 0 ? kEmpty : v;
  }
  row_plane_fit<S>(pts, r, k, l, out + kPlaneFloats * q);
}

// Launch the fit for the rows of one query call (k <= 64).
inline hipError_t launch_plane_fit(const float4 *pts, const int32_t *idx, const float4 *qs,
                                   int64_t nq, int k, float *out, hipStream_t s) {
  const uint32_t blocks = (uint32_t)((nq + 15) / 16);
  if (k <= 16)
    hipLaunchKernelGGL(plane_fit_kernel<1>, dim3(blocks), dim3(256), 0, s, pts, idx, qs, nq, k, out);
  else if (k <= 32)
    hipLaunchKernelGGL(plane_fit_kernel<2>, dim3(blocks), dim3(256), 0, s, pts, idx, qs, nq, k, out);
  else if (k <= 48)
    hipLaunchKernelGGL(plane_fit_kernel<3>, dim3(blocks), dim3(256), 0, s, pts, idx, qs, nq, k, out);
  else
    hipLaunchKernelGGL(plane_fit_kernel<4>, dim3(blocks), dim3(256), 0, s, pts, idx, qs, nq, k, out);
  return hipGetLastError();
}

}  // namespace mknn
