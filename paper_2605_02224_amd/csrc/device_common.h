// Helpers shared by the HIP translation units (plain queries and batched queries).
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "cloud.h"
#include "knn_kernels.h"

namespace mknn {

#define HIP_TRY(expr, what)                                                             \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return set_error(MKNN_EHIP, std::string(what) + ": " + hipGetErrorName(e_) + " (" + \
                                      hipGetErrorString(e_) + ")");                     \
  } while (0)

// ---- Morton codes over a bounding box (query bucketing and list placement)
struct BoxArgs {
  float lo[3], scale[3];   // scale maps the box extent to [0, 1024)
};

__host__ __device__ __forceinline__ uint32_t spread3(uint32_t v) {   // 10 bits -> every 3rd bit
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// 30-bit Morton code of a point, clamped into the box
__host__ __device__ __forceinline__ uint32_t morton30(float x, float y, float z,
                                                      const BoxArgs &b) {
  const float t[3] = {(x - b.lo[0]) * b.scale[0], (y - b.lo[1]) * b.scale[1],
                      (z - b.lo[2]) * b.scale[2]};
  uint32_t u[3];
  for (int i = 0; i < 3; ++i) {
    float v = t[i] < 0.f ? 0.f : (t[i] > 1023.f ? 1023.f : t[i]);
    u[i] = (uint32_t)v;
  }
  return (spread3(u[0]) << 2) | (spread3(u[1]) << 1) | spread3(u[2]);
}

inline BoxArgs box_of(const float lo[3], const float hi[3]) {
  BoxArgs b;
  for (int k = 0; k < 3; ++k) {
    float ext = hi[k] - lo[k];
    b.lo[k] = lo[k];
    b.scale[k] = ext > 0.f ? 1024.f / ext : 0.f;
  }
  return b;
}
// the box of the host points (packing) and of the lists on the device (query bucketing)
inline BoxArgs box_of(const mknn_cloud *c) { return box_of(c->lo, c->hi); }
inline BoxArgs dev_box_of(const mknn_cloud *c) { return box_of(c->dev_lo, c->dev_hi); }

// Record what the device lists now describe (after an upload or an applied update).
inline void note_device_state(mknn_cloud *c) {
  c->dev_head = c->head;
  for (int k = 0; k < 3; ++k) {
    c->dev_hxyz[k] = c->xyz[3 * (int64_t)c->head + k];
    c->dev_lo[k] = c->lo[k];
    c->dev_hi[k] = c->hi[k];
  }
  c->dev_n = c->n;
}

template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(T *p, int64_t cnt, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---- host helpers
inline int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
  }
  return cus;
}

inline mknn_status check_uploaded(const mknn_cloud *c, const char *who) {
  if (!c) return set_error(MKNN_EINVAL, std::string(who) + ": cloud is NULL");
  if (!c->d_ent || c->dev_version != c->version)
    return set_error(MKNN_EINVAL, std::string(who) + ": cloud is not uploaded (call mknn_upload)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
    return set_error(MKNN_EINVAL, std::string(who) + ": cloud lives on another device");
  return MKNN_OK;
}

inline void fill_cloud_args(const mknn_cloud *c, QueryArgs *a) {
  std::memset(a, 0, sizeof(*a));
  a->ent = (const float4 *)c->d_ent;
  a->lst = c->d_lst;
  a->head = c->dev_head;
  a->hx = c->dev_hxyz[0];
  a->hy = c->dev_hxyz[1];
  a->hz = c->dev_hxyz[2];
  a->n = c->dev_n;
}

// A list change in two steps: delete_prepare / insert_prepare edit the host lists and
// gather the rewritten list segments (or, when the arena's slack or the descriptor array
// would run out, a complete new image of the lists); apply_delta enqueues their copy and
// the descriptor switch (or the switch to a new arena) on a stream, asynchronously.  The
// delta must stay alive until the stream has executed the copies.
mknn_status delete_prepare(mknn_cloud *c, const int32_t *ranks, int64_t count, DeviceDelta *d);
mknn_status insert_prepare(mknn_cloud *c, const float *xyz, int64_t count, DeviceDelta *d);
mknn_status apply_delta(mknn_cloud *c, DeviceDelta *d, hipStream_t s);
// Applies a cloud's pending (lazy) deletions, and `more` ranks with them (synchronises s).
mknn_status flush_pending(mknn_cloud *c, hipStream_t s, const int32_t *more = nullptr,
                          int64_t nmore = 0);
// The server's batched run: request r filters the marks of epochs 1 .. epochs[r] of its
// cloud's epoch array (none if 0).  batch_plan_overflow: the per-request counts of rows the
// last run could not certify (pinned; valid once the run completed; NULL if nothing was
// filtered).
mknn_status batch_plan_run_pending(mknn_batch_plan *p, const mknn_request *reqs, int32_t nreq,
                                   hipStream_t s, const uint32_t *epochs);
// Marks ranks[0 .. count) (host) with `epoch` in the cloud's epoch array on stream s
// (asynchronous; the ranks are staged in a stream-ordered allocation).
mknn_status mark_deleted_async(mknn_cloud *c, const int32_t *ranks, int64_t count,
                               uint32_t epoch, hipStream_t s);
// Makes the cloud's epoch array hold at least `need` entries (new entries 0), enqueued on s.
// A replaced array is returned in *old for the caller to free once no work reads it.
mknn_status ensure_epochs_async(mknn_cloud *c, int64_t need, hipStream_t s, uint32_t **old);
const uint32_t *batch_plan_overflow(const mknn_batch_plan *p);
// After a re-pack, the replaced arena is freed by the caller once no work reads it.
void release_old_arena(DeviceDelta *d);
mknn_status pack_lists(mknn_cloud *c, HostPack *p);
mknn_status install_pack(mknn_cloud *c, const HostPack *p, hipStream_t s);
extern "C" mknn_status mknn_upload(mknn_cloud *c, void *stream);

// A launch configuration of the query kernels (see mknn_device.hip).
struct TuneConfig {
  int32_t family;      // 1 lane per query, 2 lockstep rows, 3 scheduled rows
  int32_t merge_min;   // k <= 16: candidates per chunk from which the merge network is used
  int32_t per_wave;    // row kernel: queries per wavefront
};
TuneConfig config_for(int kmax, bool exact, int64_t n);

// Optional HIP-event timing of the main query kernels (defined in mknn_device.hip).
hipError_t timing_mark(hipStream_t s, bool start);
bool timing_enabled();

}  // namespace mknn
