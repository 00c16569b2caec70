// Conversion of a float32 tensor into a narrower storage format (the paper's
// Sec. 5.5 stores tensors narrow and promotes before arithmetic).
//   TVC_F16   IEEE binary16, round to nearest even (hardware conversion).
//   TVC_BF16  round to nearest even on the bit pattern, or truncation (the
//             paper's own conversion) with TVC_QUANT_TRUNCATE.
//   TVC_F8E4M3  OCP E4M3FN with one float32 scale per mode-0 slice:
//             s_i = absmax(A[i, ...]) / 448 (1 for an all-zero slice), codes
//             = e4m3(A / s_i) rounded to nearest even, finite overflow
//             saturated to +-448.  The encoder is written from the format
//             definition so that the codes are exact and reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "common.h"
#include "internal.h"

namespace tvc {

__device__ __forceinline__ uint16_t bf16_rne(float v) {
  const uint32_t b = __float_as_uint(v);
  if (isnan(v)) return (uint16_t)(((b >> 16) & 0x8000u) | 0x7fc0u);
  const uint32_t lsb = (b >> 16) & 1u;
  return (uint16_t)((b + 0x7fffu + lsb) >> 16);
}

__device__ __forceinline__ uint8_t e4m3_rne_sat(float v) {
  const uint32_t sign = (__float_as_uint(v) >> 24) & 0x80u;
  const float a = fabsf(v);
  if (isnan(v)) return (uint8_t)(sign | 0x7fu);
  if (a >= 448.f) return (uint8_t)(sign | 0x7eu);
  if (a < 0.015625f) {                       // below 2^-6: multiples of 2^-9
    return (uint8_t)(sign | (uint32_t)rintf(a * 512.f));
  }
  int e;
  const float m = frexpf(a, &e);             // a = m 2^e, m in [0.5, 1)
  int E = e - 1;                             // a = (2m) 2^E
  int q = (int)rintf((2.f * m - 1.f) * 8.f);
  if (q == 8) {
    E += 1;
    q = 0;
  }
  return (uint8_t)(sign | (uint32_t)(((E + 7) << 3) | q));
}

__global__ void k_to_f16(const float* s, uint16_t* d, i64 n) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    d[i] = __builtin_bit_cast(uint16_t, (_Float16)s[i]);
}

__global__ void k_to_bf16(const float* s, uint16_t* d, i64 n, int trunc) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    d[i] = trunc ? (uint16_t)(__float_as_uint(s[i]) >> 16) : bf16_rne(s[i]);
}

__global__ void k_zero_u32(uint32_t* p, i64 n) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Per-slice absmax as float bits (non-negative floats order like integers, so
// an integer max is exact and order-independent).
__global__ __launch_bounds__(kBlock) void k_absmax(const float* s, i64 slab, i64 chunk,
                                                   i64 chunks_per_slab, uint32_t* amax,
                                                   i64 ntasks) {
  __shared__ uint32_t sh[kBlock / kWave];
  for (i64 t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const i64 i0 = t / chunks_per_slab;
    const i64 c = t % chunks_per_slab;
    const i64 b = i0 * slab + c * chunk;
    const i64 e = i0 * slab + min(slab, (c + 1) * chunk);
    uint32_t m = 0u;
    for (i64 i = b + threadIdx.x; i < e; i += kBlock) {
      const float a = fabsf(s[i]);
      const uint32_t u = isnan(a) ? 0u : __float_as_uint(a);
      m = max(m, u);
    }
    for (int off = kWave / 2; off >= 1; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, kWave));
    if (lane_id() == 0) sh[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t mm = 0u;
      for (int w = 0; w < kBlock / kWave; ++w) mm = max(mm, sh[w]);
      atomicMax(&amax[i0], mm);
    }
    __syncthreads();
  }
}

__global__ void k_scale_from_amax(uint32_t* p, i64 n) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
    const float a = __uint_as_float(p[i]);
    const float s = a == 0.f ? 1.f : a / 448.f;
    p[i] = __float_as_uint(s);
  }
}

__global__ void k_to_e4m3(const float* s, const float* scale, uint8_t* d, i64 n, i64 slab) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    d[i] = e4m3_rne_sat(s[i] / scale[i / slab]);
}

}  // namespace tvc

using namespace tvc;

extern "C" int32_t tvc_quantize(const tvc_tensor* src, void* dst, int32_t dst_dtype,
                                float* slab_scale_out, int32_t flags, void* stream) {
  tvc_status st = check_tensor(src, "src");
  if (st != TVC_OK) return st;
  if (src->dtype != TVC_F32) return fail(TVC_EDTYPE, "src must be TVC_F32");
  if (dst_dtype != TVC_F16 && dst_dtype != TVC_BF16 && dst_dtype != TVC_F8E4M3)
    return fail(TVC_EDTYPE, "dst_dtype must be TVC_F16, TVC_BF16 or TVC_F8E4M3");
  if (!dst) return fail(TVC_EINVAL, "dst is NULL");
  const i64 n = numel(src);
  const size_t db = (size_t)n * elem_bytes(dst_dtype);
  if ((uintptr_t)dst % elem_bytes(dst_dtype) != 0) return fail(TVC_EINVAL, "dst misaligned");
  if (overlaps(dst, db, src->data, (size_t)n * 4)) return fail(TVC_EALIAS, "dst overlaps src");
  hipStream_t s = (hipStream_t)stream;
  const int g = (int)std::max<i64>(1, std::min<i64>((n + 255) / 256, 8 * (i64)device_cus()));
  const float* a = (const float*)src->data;
  if (dst_dtype == TVC_F16) {
    hipLaunchKernelGGL(k_to_f16, dim3(g), dim3(256), 0, s, a, (uint16_t*)dst, n);
  } else if (dst_dtype == TVC_BF16) {
    hipLaunchKernelGGL(k_to_bf16, dim3(g), dim3(256), 0, s, a, (uint16_t*)dst, n,
                       (flags & TVC_QUANT_TRUNCATE) ? 1 : 0);
  } else {
    if (!slab_scale_out) return fail(TVC_EINVAL, "slab_scale_out is NULL");
    if ((uintptr_t)slab_scale_out % 4 != 0) return fail(TVC_EINVAL, "slab_scale_out misaligned");
    const i64 n0 = src->dims[0];
    if (overlaps(slab_scale_out, (size_t)n0 * 4, src->data, (size_t)n * 4) ||
        overlaps(slab_scale_out, (size_t)n0 * 4, dst, db))
      return fail(TVC_EALIAS, "slab_scale_out overlaps src or dst");
    const i64 slab = n / n0;
    uint32_t* am = (uint32_t*)slab_scale_out;
    const int g0 = (int)std::max<i64>(1, std::min<i64>((n0 + 255) / 256, 1024));
    hipLaunchKernelGGL(k_zero_u32, dim3(g0), dim3(256), 0, s, am, n0);
    const i64 chunk = 1 << 16;
    const i64 cps = (slab + chunk - 1) / chunk;
    const i64 tasks = n0 * cps;
    const int ga = (int)std::max<i64>(1, std::min<i64>(tasks, 8 * (i64)device_cus()));
    hipLaunchKernelGGL(k_absmax, dim3(ga), dim3(kBlock), 0, s, a, slab, chunk, cps, am, tasks);
    hipLaunchKernelGGL(k_scale_from_amax, dim3(g0), dim3(256), 0, s, am, n0);
    hipLaunchKernelGGL(k_to_e4m3, dim3(g), dim3(256), 0, s, a, (const float*)slab_scale_out,
                       (uint8_t*)dst, n, slab);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TVC_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
  return TVC_OK;
}
