// Internal device helpers shared by the HIP kernels of libtvc (gfx950 only).
//
// Storage formats and their promotion before arithmetic (the paper's
// mixed-precision scheme, Sec. 5.5: low precision is a storage format only):
//   TVC_F64 -> double accumulate;  TVC_F32, TVC_F16, TVC_BF16, TVC_F8E4M3 ->
//   float accumulate.  A "unit" is one 16-byte vector load (EPV elements) on
//   the vector paths, or one element on the scalar paths.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tvc.h"

namespace tvc {

typedef int64_t i64;

constexpr int kWave = 64;      // CDNA wavefront width
constexpr int kBlock = 256;    // threads per workgroup for the streaming kernels

template <int DT> struct St;
template <> struct St<TVC_F64>    { typedef double   T; typedef double Acc; static constexpr int EPV = 2; };
template <> struct St<TVC_F32>    { typedef float    T; typedef float  Acc; static constexpr int EPV = 4; };
template <> struct St<TVC_F16>    { typedef uint16_t T; typedef float  Acc; static constexpr int EPV = 8; };
template <> struct St<TVC_BF16>   { typedef uint16_t T; typedef float  Acc; static constexpr int EPV = 8; };
template <> struct St<TVC_F8E4M3> { typedef uint8_t  T; typedef float  Acc; static constexpr int EPV = 16; };

// ---------------------------------------------------------------- conversions
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ float f16_bits(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(h & 0xffffu));
}
// gfx950 converts OCP E4M3 in hardware: two bytes of a dword per instruction.
__device__ __forceinline__ void e4m3x4(uint32_t w, float* o) {
  auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
  o[0] = lo[0]; o[1] = lo[1]; o[2] = hi[0]; o[3] = hi[1];
}
__device__ __forceinline__ float e4m3_one(uint32_t b) {
  return __builtin_amdgcn_cvt_f32_fp8((int)(b & 0xffu), 0);
}

// One element, promoted.
template <int DT> __device__ __forceinline__ typename St<DT>::Acc load_elem(const void* p, i64 i);
template <> __device__ __forceinline__ double load_elem<TVC_F64>(const void* p, i64 i) { return ((const double*)p)[i]; }
template <> __device__ __forceinline__ float load_elem<TVC_F32>(const void* p, i64 i) { return ((const float*)p)[i]; }
template <> __device__ __forceinline__ float load_elem<TVC_F16>(const void* p, i64 i) { return f16_bits(((const uint16_t*)p)[i]); }
template <> __device__ __forceinline__ float load_elem<TVC_BF16>(const void* p, i64 i) { return bf16_lo(((const uint16_t*)p)[i]); }
template <> __device__ __forceinline__ float load_elem<TVC_F8E4M3>(const void* p, i64 i) { return e4m3_one(((const uint8_t*)p)[i]); }

// One 16-byte vector, promoted into EPV values.
template <int DT> __device__ __forceinline__ void unpack16(const uint4& r, typename St<DT>::Acc* o);
template <> __device__ __forceinline__ void unpack16<TVC_F64>(const uint4& r, double* o) {
  o[0] = __hiloint2double((int)r.y, (int)r.x);
  o[1] = __hiloint2double((int)r.w, (int)r.z);
}
template <> __device__ __forceinline__ void unpack16<TVC_F32>(const uint4& r, float* o) {
  o[0] = __uint_as_float(r.x); o[1] = __uint_as_float(r.y);
  o[2] = __uint_as_float(r.z); o[3] = __uint_as_float(r.w);
}
template <> __device__ __forceinline__ void unpack16<TVC_BF16>(const uint4& r, float* o) {
  o[0] = bf16_lo(r.x); o[1] = bf16_hi(r.x); o[2] = bf16_lo(r.y); o[3] = bf16_hi(r.y);
  o[4] = bf16_lo(r.z); o[5] = bf16_hi(r.z); o[6] = bf16_lo(r.w); o[7] = bf16_hi(r.w);
}
template <> __device__ __forceinline__ void unpack16<TVC_F16>(const uint4& r, float* o) {
  o[0] = f16_bits(r.x); o[1] = f16_bits(r.x >> 16); o[2] = f16_bits(r.y); o[3] = f16_bits(r.y >> 16);
  o[4] = f16_bits(r.z); o[5] = f16_bits(r.z >> 16); o[6] = f16_bits(r.w); o[7] = f16_bits(r.w >> 16);
}
template <> __device__ __forceinline__ void unpack16<TVC_F8E4M3>(const uint4& r, float* o) {
  e4m3x4(r.x, o); e4m3x4(r.y, o + 4); e4m3x4(r.z, o + 8); e4m3x4(r.w, o + 12);
}

// One dword of a narrow format, promoted: 2 fp16 / bf16 or 4 E4M3 values
// (low bits first).
template <int DT> __device__ __forceinline__ void unpack4(uint32_t w, float* o);
template <> __device__ __forceinline__ void unpack4<TVC_BF16>(uint32_t w, float* o) { o[0] = bf16_lo(w); o[1] = bf16_hi(w); }
template <> __device__ __forceinline__ void unpack4<TVC_F16>(uint32_t w, float* o) { o[0] = f16_bits(w); o[1] = f16_bits(w >> 16); }
template <> __device__ __forceinline__ void unpack4<TVC_F8E4M3>(uint32_t w, float* o) { e4m3x4(w, o); }

// 16-byte vectors that need only dword alignment.  Multi-dword global
// accesses on CDNA need a dword-aligned address, not a 16-byte-aligned one,
// so rows whose length is not a whole number of 16-byte vectors (odd
// extents in float32, say) still stream as dwordx4 loads and stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4), aligned(4)));
// 16 bytes at any byte address: global loads on gfx950 need no alignment
// (rows of 1- and 2-byte formats of odd length start on any byte)
typedef unsigned int u32x4u __attribute__((ext_vector_type(4), aligned(1)));

// Streaming loads of A use the nontemporal hint: every element is read once,
// so it should not displace the vectors, weights and partial sums that are
// reused from the caches (measured on gfx950: about 15% more read bandwidth).
#ifndef TVC_NT_LOADS
#define TVC_NT_LOADS 1
#endif

__device__ __forceinline__ uint4 stream_load16(const void* p) {
#if TVC_NT_LOADS
  const u32x4u v = __builtin_nontemporal_load((const u32x4u*)p);
#else
  const u32x4u v = *(const u32x4u*)p;
#endif
  uint4 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
#if TVC_NT_LOADS
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// A unit: VEC -> 16 bytes (EPV elements) at a dword-aligned address;
// scalar -> one element.  Units are addressed by their first element.
template <int DT, bool VEC> struct Unit {
  static constexpr int EU = VEC ? St<DT>::EPV : 1;
  typedef typename St<DT>::Acc Acc;
  typedef typename St<DT>::T T;
  typedef typename std::conditional<VEC, uint4, T>::type Raw;
  __device__ __forceinline__ static Raw load(const void* base, i64 e) {
    if constexpr (VEC) {
      return stream_load16((const T*)base + e);
    } else {
      return stream_load((const T*)base + e);
    }
  }
  __device__ __forceinline__ static Raw zero() { Raw r; __builtin_memset(&r, 0, sizeof(Raw)); return r; }
  __device__ __forceinline__ static void unpack(const Raw& r, Acc* o) {
    if constexpr (VEC) {
      unpack16<DT>(r, o);
    } else {
      o[0] = load_elem<DT>(&r, 0);
    }
  }
};

// EU consecutive weights starting at element e (dword-aligned vector loads
// when they span whole 16-byte vectors).
template <typename Acc, int EU>
__device__ __forceinline__ void load_w(const Acc* w, i64 e, Acc* o) {
  if constexpr (EU * sizeof(Acc) >= 16) {
    const u32x4* p = (const u32x4*)(w + e);
#pragma unroll
    for (int q = 0; q < (int)(EU * sizeof(Acc) / 16); ++q) {
      const u32x4 r = p[q];
      if constexpr (sizeof(Acc) == 4) {
        o[4 * q + 0] = __uint_as_float(r.x); o[4 * q + 1] = __uint_as_float(r.y);
        o[4 * q + 2] = __uint_as_float(r.z); o[4 * q + 3] = __uint_as_float(r.w);
      } else {
        o[2 * q + 0] = __hiloint2double((int)r.y, (int)r.x);
        o[2 * q + 1] = __hiloint2double((int)r.w, (int)r.z);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < EU; ++q) o[q] = w[e + q];
  }
}

// EU consecutive values to dst (dword-aligned vector stores when they span
// whole 16-byte vectors).
template <typename Acc, int EU>
__device__ __forceinline__ void store_w(Acc* dst, const Acc* v) {
  if constexpr ((EU * sizeof(Acc)) % 16 == 0) {
#pragma unroll
    for (int q = 0; q < (int)(EU * sizeof(Acc) / 16); ++q) {
      u32x4 u;
      __builtin_memcpy(&u, v + q * (16 / sizeof(Acc)), 16);
      ((u32x4*)dst)[q] = u;
    }
  } else {
#pragma unroll
    for (int e = 0; e < EU; ++e) dst[e] = v[e];
  }
}

// ---------------------------------------------------------------- reductions
template <typename Acc>
__device__ __forceinline__ Acc shfl_xor(Acc v, int m) {
  return __shfl_xor(v, m, kWave);
}

template <typename Acc>
__device__ __forceinline__ Acc wave_sum(Acc v) {
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) v += shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// A lane permutation within each row of 16 lanes (a DPP operand modifier:
// no LDS traffic, a few cycles).  CTRL: 0xB1 swaps neighbouring lanes,
// 0x4E swaps neighbouring pairs, 0x141 mirrors each half-row of 8 lanes,
// 0x140 mirrors the row.
template <int CTRL>
__device__ __forceinline__ float dpp_perm(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_perm(double v) {
  const uint64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Sum over aligned groups of 2^glog lanes (glog <= 6); every lane of a group
// gets its group's sum, added in the same order in every group.  Within a
// row of 16 lanes the partners come from DPP permutations (after the first
// two steps each group of 4 holds its sum, which the half-row mirror pairs
// with the neighbouring group of 4, and the row mirror pairs halves); 32-
// and 64-lane groups finish with two cross-row shuffles.
template <typename Acc>
__device__ __forceinline__ Acc group_sum(Acc v, int glog) {
  if (glog >= 1) v += dpp_perm<0xB1>(v);
  if (glog >= 2) v += dpp_perm<0x4E>(v);
  if (glog >= 3) v += dpp_perm<0x141>(v);
  if (glog >= 4) v += dpp_perm<0x140>(v);
  if (glog >= 5) v += shfl_xor(v, 16);
  if (glog >= 6) v += shfl_xor(v, 32);
  return v;
}

// q = a / b, r = a mod b for non-negative a, b > 0: 32-bit division when
// both fit (task and row indices almost always do), 64-bit otherwise.
__device__ __forceinline__ void divmod(i64 a, i64 b, i64& q, i64& r) {
  if ((((uint64_t)a | (uint64_t)b) >> 32) == 0) {
    const uint32_t qq = (uint32_t)a / (uint32_t)b;
    q = qq;
    r = (uint32_t)a - qq * (uint32_t)b;
  } else {
    q = a / b;
    r = a - q * b;
  }
}

}  // namespace tvc
