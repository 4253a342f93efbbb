// Memory probes for the roofline of the query kernels: the sustained rate of a streaming
// read and of random 16-byte record gathers (the access pattern of a list walk that opens a
// new list at every step), measured on the caller's buffer with HIP events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "device_common.h"

namespace mknn {

// Streaming read: every thread reads float4 records with a grid-stride loop, four
// independent loads in flight.  The sum is written only if `sink_on` is set (never, in
// practice); the loads cannot be removed because the flag is a runtime value.
__global__ __launch_bounds__(256) void probe_stream_kernel(const float4 *buf, int64_t n4,
                                                           float *sink, int32_t sink_on) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const float4 v0 = buf[i], v1 = buf[i + stride], v2 = buf[i + 2 * stride], v3 = buf[i + 3 * stride];
    a0 += v0.x + v0.y + v0.z + v0.w;
    a1 += v1.x + v1.y + v1.z + v1.w;
    a2 += v2.x + v2.y + v2.z + v2.w;
    a3 += v3.x + v3.y + v3.z + v3.w;
  }
  for (; i < n4; i += stride) {
    const float4 v = buf[i];
    a0 += v.x + v.y + v.z + v.w;
  }
  if (sink_on) sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = (a0 + a1) + (a2 + a3);
}

// Random gather: thread t reads `per_thread` 16-byte records at indices given by a
// multiplicative hash of (t, j), masked to the power-of-two record count n4.
__global__ __launch_bounds__(256) void probe_gather_kernel(const float4 *buf, uint64_t mask,
                                                           int32_t per_thread, float *sink,
                                                           int32_t sink_on) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float a0 = 0.f, a1 = 0.f;
  uint64_t h = (t + 1) * 0x9E3779B97F4A7C15ull;
  for (int32_t j = 0; j < per_thread; j += 2) {
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    const uint64_t i0 = (h >> 11) & mask;
    h ^= h >> 32;
    h *= 0x94D049BB133111EBull;
    const uint64_t i1 = (h >> 11) & mask;
    const float4 v0 = buf[i0], v1 = buf[i1];
    a0 += v0.x + v0.y + v0.z + v0.w;
    a1 += v1.x + v1.y + v1.z + v1.w;
  }
  if (sink_on) sink[t] = a0 + a1;
}

// Best rate over `reps` timed launches (after one untimed one), in GB/s of useful bytes.
template <typename Launch>
static mknn_status time_best(Launch launch, double bytes, int32_t reps, hipStream_t s,
                             const char *who, double *gbps) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = INFINITY;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && r > 0) best = std::min(best, ms);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return set_error(MKNN_EHIP, std::string(who) + ": " + hipGetErrorName(e));
  *gbps = bytes / (best * 1e-3) / 1e9;
  return MKNN_OK;
}

}  // namespace mknn

using namespace mknn;

extern "C" {

mknn_status mknn_probe_stream_read(const void *d_buf, int64_t bytes, int32_t reps, void *stream,
                                   double *gbps) {
  clear_error();
  if (!d_buf || !gbps || bytes < 16 * 256 || (bytes & 15) || reps < 1)
    return set_error(MKNN_EINVAL, "mknn_probe_stream_read: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n4 = bytes / 16;
  const uint32_t blocks = (uint32_t)std::min<int64_t>((int64_t)device_cus() * 32, (n4 + 255) / 256);
  auto launch = [&]() {
    hipLaunchKernelGGL(probe_stream_kernel, dim3(blocks), dim3(256), 0, s, (const float4 *)d_buf,
                       n4, (float *)nullptr, 0);
    return hipGetLastError();
  };
  return time_best(launch, (double)n4 * 16.0, reps, s, "mknn_probe_stream_read", gbps);
}

mknn_status mknn_probe_gather16(const void *d_buf, int64_t bytes, int64_t accesses, int32_t reps,
                                void *stream, double *gbps) {
  clear_error();
  if (!d_buf || !gbps || bytes < 16 * 256 || reps < 1 || accesses < 1)
    return set_error(MKNN_EINVAL, "mknn_probe_gather16: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  uint64_t n4 = 1;
  while (n4 * 2 * 16 <= (uint64_t)bytes) n4 *= 2;   // power-of-two record count in the buffer
  const int32_t per_thread = 64;
  const int64_t threads = std::max<int64_t>(256, (accesses + per_thread - 1) / per_thread);
  const uint32_t blocks = (uint32_t)((threads + 255) / 256);
  auto launch = [&]() {
    hipLaunchKernelGGL(probe_gather_kernel, dim3(blocks), dim3(256), 0, s, (const float4 *)d_buf,
                       (uint64_t)(n4 - 1), per_thread, (float *)nullptr, 0);
    return hipGetLastError();
  };
  return time_best(launch, (double)blocks * 256.0 * per_thread * 16.0, reps, s,
                   "mknn_probe_gather16", gbps);
}

}  // extern "C"
