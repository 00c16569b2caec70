// Bandwidth probes: the library's own yardstick for achievable HBM bandwidth
// (the role STREAM plays in the paper's Sec. 5.1), with the same 16-byte
// loads and persistent grid-stride pattern as the contraction kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "common.h"
#include "internal.h"

namespace tvc {

constexpr int kProbeUnroll = 8;

// Sum of every float of `src` per workgroup (keeps the loads live).
__global__ __launch_bounds__(kBlock) void k_probe_read(const uint4* src, i64 units, float* sink) {
  float acc = 0.f;
  const i64 stride = (i64)gridDim.x * kBlock;
  i64 u = (i64)blockIdx.x * kBlock + threadIdx.x;
  for (; u + (kProbeUnroll - 1) * stride < units; u += kProbeUnroll * stride) {
    uint4 r[kProbeUnroll];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) r[k] = src[u + k * stride];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k)
      acc += __uint_as_float(r[k].x) + __uint_as_float(r[k].y) + __uint_as_float(r[k].z) +
             __uint_as_float(r[k].w);
  }
  for (; u < units; u += stride) {
    uint4 r = src[u];
    acc += __uint_as_float(r.x) + __uint_as_float(r.y) + __uint_as_float(r.z) + __uint_as_float(r.w);
  }
  acc = wave_sum(acc);
  __shared__ float part[kBlock / kWave];
  if (lane_id() == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < kBlock / kWave; ++i) s += part[i];
    sink[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_probe_copy(const uint4* src, uint4* dst, i64 units) {
  const i64 stride = (i64)gridDim.x * kBlock;
  i64 u = (i64)blockIdx.x * kBlock + threadIdx.x;
  for (; u + (kProbeUnroll - 1) * stride < units; u += kProbeUnroll * stride) {
    uint4 r[kProbeUnroll];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) r[k] = src[u + k * stride];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) dst[u + k * stride] = r[k];
  }
  for (; u < units; u += stride) dst[u] = src[u];
}

}  // namespace tvc

using namespace tvc;

extern "C" {

int32_t tvc_probe_read(const void* src, size_t bytes, float* sink, int32_t grid, void* stream) {
  if (!src || !sink) return fail(TVC_EINVAL, "NULL pointer");
  if (bytes % 16 != 0 || (uintptr_t)src % 16 != 0)
    return fail(TVC_EINVAL, "bytes and src must be multiples of 16");
  if (grid <= 0) grid = 8 * device_cus();
  hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                     (const uint4*)src, (i64)(bytes / 16), sink);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TVC_EHIP, hipGetErrorString(e));
  return TVC_OK;
}

int32_t tvc_probe_copy(const void* src, void* dst, size_t bytes, int32_t grid, void* stream) {
  if (!src || !dst) return fail(TVC_EINVAL, "NULL pointer");
  if (bytes % 16 != 0 || (uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0)
    return fail(TVC_EINVAL, "bytes and pointers must be multiples of 16");
  if (overlaps(src, bytes, dst, bytes)) return fail(TVC_EALIAS, "src and dst overlap");
  if (grid <= 0) grid = 8 * device_cus();
  hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                     (const uint4*)src, (uint4*)dst, (i64)(bytes / 16));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TVC_EHIP, hipGetErrorString(e));
  return TVC_OK;
}

}  // extern "C"
