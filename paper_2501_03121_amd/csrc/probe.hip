// Bandwidth probes: the library's own yardstick for achievable HBM bandwidth
// (the role STREAM plays in the paper's Sec. 5.1): the access pattern that
// reads fastest on this part (nontemporal 16-byte loads, each workgroup
// streaming one contiguous range), so that the contraction kernels can be
// set against the achievable read rate as well as the 8 TB/s specification.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "common.h"
#include "internal.h"

namespace tvc {

constexpr int kProbeUnroll = 8;

// Units [b, e) of workgroup blockIdx.x: one contiguous range per workgroup,
// consecutive workgroups on consecutive ranges.
__device__ __forceinline__ void probe_range(i64 units, i64& b, i64& e) {
  const i64 per = (units + gridDim.x - 1) / gridDim.x;
  b = (i64)blockIdx.x * per;
  e = b + per < units ? b + per : units;
}

// Sum of every float of `src` per workgroup (keeps the loads live).  Each
// workgroup streams its own contiguous range with nontemporal 16-byte loads,
// kProbeUnroll in flight per thread; a wave load covers 1 KB.
__global__ __launch_bounds__(kBlock) void k_probe_read(const uint4* src, i64 units, float* sink) {
  i64 b, e;
  probe_range(units, b, e);
  float acc = 0.f;
  i64 u = b + threadIdx.x;
  for (; u + (kProbeUnroll - 1) * kBlock < e; u += kProbeUnroll * kBlock) {
    uint4 r[kProbeUnroll];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) r[k] = stream_load16(src + u + k * kBlock);
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k)
      acc += __uint_as_float(r[k].x) + __uint_as_float(r[k].y) + __uint_as_float(r[k].z) +
             __uint_as_float(r[k].w);
  }
  for (; u < e; u += kBlock) {
    const uint4 r = stream_load16(src + u);
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

__device__ __forceinline__ void stream_store16(uint4* p, const uint4& r) {
  u32x4 v;
  __builtin_memcpy(&v, &r, 16);
  __builtin_nontemporal_store(v, (u32x4*)p);
}

// Copy with the same pattern; nontemporal stores.
__global__ __launch_bounds__(kBlock) void k_probe_copy(const uint4* src, uint4* dst, i64 units) {
  i64 b, e;
  probe_range(units, b, e);
  i64 u = b + threadIdx.x;
  for (; u + (kProbeUnroll - 1) * kBlock < e; u += kProbeUnroll * kBlock) {
    uint4 r[kProbeUnroll];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) r[k] = stream_load16(src + u + k * kBlock);
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) stream_store16(dst + u + k * kBlock, r[k]);
  }
  for (; u < e; u += kBlock) stream_store16(dst + u, stream_load16(src + u));
}

}  // namespace tvc

using namespace tvc;

extern "C" {

int32_t tvc_probe_read(const void* src, size_t bytes, float* sink, int32_t grid, void* stream) {
  if (!src || !sink) return fail(TVC_EINVAL, "NULL pointer");
  if (bytes % 16 != 0 || (uintptr_t)src % 16 != 0)
    return fail(TVC_EINVAL, "bytes and src must be multiples of 16");
  if (grid <= 0) grid = 4 * device_cus();
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
  if (grid <= 0) grid = 4 * device_cus();
  hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                     (const uint4*)src, (uint4*)dst, (i64)(bytes / 16));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TVC_EHIP, hipGetErrorString(e));
  return TVC_OK;
}

}  // extern "C"
