// Derivatives of the k-mode contraction Y = A x_k x (Sec. 3 definition, on
// the [L][M][R] view) and the dense rank-R update used to materialise the
// gradient of unrolled HOPM sweeps.
//
//   dx[m]    = sum_{l, r} A[l, m, r] g[l, r]     (a reduction of all of A
//              into n_k values: HBM-bound, one pass over A)
//   dA       = alpha * g (x)_k x + beta * dA     (write-bound outer product)
//   D        = alpha * A + sum_r c_r f_{r,0} o ... o f_{r,d-1}
//              (split into rows = modes [0, h) and columns = modes [h, d):
//              a K = R product of two thin factor matrices, tiled through
//              LDS, with the alpha * A epilogue fused)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "common.h"
#include "internal.h"

namespace tvc {

namespace {

__host__ __device__ inline i64 cdiv_(i64 a, i64 b) { return (a + b - 1) / b; }

int grid_(i64 blocks, int per_cu = 8) {
  return (int)std::max<i64>(1, std::min<i64>(blocks, (i64)per_cu * device_cus()));
}

}  // namespace

// w[l] = g[l] * scale[l / div]
__global__ void k_scale_rows(const float* g, const float* scale, i64 div, float* w, i64 n) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    w[i] = g[i] * scale[i / div];
}

template <typename Acc>
__global__ void k_fill(Acc* p, i64 n, Acc v) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    p[i] = v;
}

// dA written as rows: row i (length n) holds
//     alpha * s[i mod smod] * v[(i / vdiv) * n + c]  (+ beta * dA)
// For R > 1 the rows are the (l, m) rows of the [L*M][R] view (s = x with
// smod = M, v = g with vdiv = M); for R == 1 they are the l rows of the
// [L][M] view (s = g, v = x shared by every row).  G lanes per row (a power
// of two, at most 64), P = 64/G rows per wave step; rows longer than a wave
// are cut into chunks of `chunk` units so that enough waves write at once.
// Per row one index division; 16-byte nontemporal stores at dword alignment,
// the ragged end of a row stored element by element.
template <typename Acc, bool VEC, bool BETA, bool BLOCKED>
__global__ __launch_bounds__(kBlock) void k_outer_rows(const Acc* sv, i64 smod, const Acc* v, i64 vdiv,
                                                        Acc* out, i64 rows, i64 n, i64 upr, int tail,
                                                        int glog, i64 chunk, i64 nch, Acc alpha,
                                                        Acc beta) {
  constexpr int EU = VEC ? (int)(16 / sizeof(Acc)) : 1;
  const int lane = lane_id();
  const int G = 1 << glog, P = kWave >> glog;
  const int sub = lane & (G - 1), rsub = lane >> glog;
  const i64 nu = upr + (tail > 0 ? 1 : 0);
  // With BLOCKED (rows of several chunks) the task order is (chunk block,
  // row group, chunk within the block): waves at work together cover a
  // block of up to 16 chunks of many rows, so a row of v shared by many
  // rows (mode 0: one row of g for every output row) is read from HBM once
  // per block and served from the L2 after that.
  const i64 nrt = (rows + P - 1) / P;
  const i64 cb = nch < 16 ? nch : 16;
  const i64 tasks = BLOCKED ? (nch + cb - 1) / cb * nrt * cb : nrt * nch;
  constexpr int wpb = kBlock / kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (i64 t = (i64)blockIdx.x * wpb + w; t < tasks; t += (i64)gridDim.x * wpb) {
    i64 rt, ch;
    if constexpr (BLOCKED) {
      i64 bq, ci, bb;
      divmod(t, cb, bq, ci);
      divmod(bq, nrt, bb, rt);
      ch = bb * cb + ci;
      if (ch >= nch) continue;
    } else {
      divmod(t, nch, rt, ch);
    }
    const i64 row = rt * P + rsub;
    if (row >= rows) continue;
    i64 vq, vr, sq, sr;
    divmod(row, smod, sq, sr);
    divmod(row, vdiv, vq, vr);
    const Acc sc = alpha * sv[sr];
    const Acc* vrow = v + vq * n;
    Acc* orow = out + row * n;
    const i64 u1 = min(nu, (ch + 1) * chunk);
    for (i64 u = ch * chunk + sub; u < u1; u += G) {
      const bool tl = tail > 0 && u == upr;
      const i64 e = tl ? n - EU : u * EU;
      Acc gv[EU], o[EU];
      load_w<Acc, EU>(vrow, e, gv);
      if constexpr (BETA) load_w<Acc, EU>(orow + e, 0, o);
#pragma unroll
      for (int q = 0; q < EU; ++q) o[q] = BETA ? fma(gv[q], sc, beta * o[q]) : gv[q] * sc;
      if (!tl) {
        if constexpr (VEC) {
          u32x4 st;
          __builtin_memcpy(&st, o, 16);
          __builtin_nontemporal_store(st, (u32x4*)(orow + e));
        } else {
          orow[e] = o[0];
        }
      } else {
#pragma unroll
        for (int q = 0; q < EU; ++q)
          if (q >= EU - tail) orow[e + q] = o[q];
      }
    }
  }
}

// ---------------------------------------------------------------- rank update
// P[r][row] = c_r * prod_{k < h} f_{r,k}[i_k],  Q[r][col] = prod_{k >= h} f_{r,k}[i_k]
struct FactorArgs {
  int h, d;
  i64 dims[TVC_MAX_ORDER];
  i64 offs[TVC_MAX_ORDER];
  i64 nsum;
};

template <typename T>
__global__ void k_factor_rows(const double* f, const double* coef, FactorArgs fa, int R, T* P,
                              i64 rows, int first, int last, int with_coef) {
  const i64 total = (i64)R * rows;
  for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (i64)gridDim.x * blockDim.x) {
    const i64 r = t / rows;
    i64 rem = t - r * rows;
    double p = with_coef ? coef[r] : 1.0;
    for (int k = last - 1; k >= first; --k) {
      const i64 i = rem % fa.dims[k];
      rem /= fa.dims[k];
      p *= f[r * fa.nsum + fa.offs[k] + i];
    }
    P[t] = (T)p;
  }
}

constexpr int kTileR = 64;    // rows per workgroup tile
constexpr int kTileC = 64;    // columns per workgroup tile
constexpr int kTileK = 16;    // factor terms staged per LDS round

// D[row, col] = alpha * A[row, col] + sum_r P[r][row] * Q[r][col]; 16 x 16
// threads, each owning a 4 x 4 block of outputs.
template <typename T, bool HAS_A>
__global__ __launch_bounds__(256) void k_rank_update(const T* A, T alpha, const T* P,
                                                     const T* Q, int R, i64 rows, i64 cols,
                                                     T* D) {
  __shared__ T sp[kTileK][kTileR];
  __shared__ T sq[kTileK][kTileC];
  const int tx = threadIdx.x % 16;   // column group
  const int ty = threadIdx.x / 16;   // row group
  const i64 ctiles = cdiv_(cols, kTileC);
  const i64 ntiles = cdiv_(rows, kTileR) * ctiles;
  for (i64 t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const i64 row0 = (t / ctiles) * kTileR;
    const i64 col0 = (t % ctiles) * kTileC;
    T acc[4][4] = {};
    for (int k0 = 0; k0 < R; k0 += kTileK) {
      for (int e = threadIdx.x; e < kTileK * kTileR; e += 256) {
        const int kk = e / kTileR, rr = e % kTileR;
        const i64 row = row0 + rr;
        sp[kk][rr] = (k0 + kk < R && row < rows) ? P[(i64)(k0 + kk) * rows + row] : (T)0;
        const i64 col = col0 + rr;
        sq[kk][rr] = (k0 + kk < R && col < cols) ? Q[(i64)(k0 + kk) * cols + col] : (T)0;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kTileK; ++kk) {
        T a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = sp[kk][ty * 4 + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = sq[kk][tx * 4 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const i64 row = row0 + ty * 4 + i;
      if (row >= rows) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const i64 col = col0 + tx * 4 + j;
        if (col >= cols) continue;
        const i64 idx = row * cols + col;
        T v = acc[i][j];
        if constexpr (HAS_A) v = fma(alpha, A[idx], v);
        D[idx] = v;
      }
    }
  }
}

namespace {

// Bytes of scratch for dx of `mode` and the plans involved.
struct BxPlan {
  i64 L, M, R;
  int kind;                 // 0: right extent 1, 1: left extent 1, 2: middle
  size_t o_w = 0, o_P = 0, o_ones = 0, o_part = 0, total = 0;
  size_t part = 0;
};

BxPlan plan_bx(const tvc_tensor* A, int mode) {
  BxPlan b;
  mode_view(A, mode, &b.L, &b.M, &b.R);
  const size_t ab = acc_bytes(A->dtype);
  const int accdt = A->dtype == TVC_F64 ? TVC_F64 : TVC_F32;
  size_t o = 0;
  auto take = [&](size_t n) { size_t at = o; o += align256(n); return at; };
  if (mode == 0) {
    b.kind = 1;
    for (int a16 = 0; a16 < 2; ++a16)
      for (int w16 = 0; w16 < 2; ++w16)
        b.part = std::max(b.part, plan_tvc(A->dtype, b.M, b.R, 1, a16, w16).part_bytes);
  } else if (b.R == 1) {
    b.kind = 0;
    if (A->dtype == TVC_F8E4M3) b.o_w = take((size_t)b.L * 4);
    for (int a16 = 0; a16 < 2; ++a16)
      b.part = std::max(b.part, plan_tvc(A->dtype, 1, b.L, b.M, a16, true).part_bytes);
  } else {
    b.kind = 2;
    b.o_P = take((size_t)(b.L * b.M) * ab);
    b.o_ones = take((size_t)b.L * ab);
    for (int a16 = 0; a16 < 2; ++a16)
      for (int w16 = 0; w16 < 2; ++w16)
        b.part = std::max(b.part, plan_rows_pw(A->dtype, b.L * b.M, b.R, a16, w16, b.M).part_bytes);
    b.part = std::max(b.part, plan_tvc(accdt, 1, b.L, b.M, true, true).part_bytes);
  }
  b.o_part = take(b.part);
  b.total = o;
  return b;
}

#define BX_TRY_HIP(expr)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(TVC_EHIP, std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

}  // namespace tvc

using namespace tvc;

extern "C" {

size_t tvc_backward_x_workspace_bytes(const tvc_tensor* A, int32_t mode) {
  if (check_tensor(A, "A") != TVC_OK || mode < 0 || mode >= A->order) return 0;
  return plan_bx(A, mode).total;
}

int32_t tvc_backward_x(const tvc_tensor* A, int32_t mode, const void* g, void* dx, void* ws,
                       size_t ws_bytes, void* stream) {
  tvc_status s = check_tensor(A, "A");
  if (s != TVC_OK) return s;
  if (mode < 0 || mode >= A->order) return fail(TVC_EINVAL, "mode outside [0, order)");
  if (!g || !dx) return fail(TVC_EINVAL, "g or dx is NULL");
  const size_t ab = acc_bytes(A->dtype);
  if ((uintptr_t)g % ab || (uintptr_t)dx % ab) return fail(TVC_EINVAL, "g or dx misaligned");
  BxPlan b = plan_bx(A, mode);
  const size_t abytes = (size_t)numel(A) * elem_bytes(A->dtype);
  if (overlaps(dx, (size_t)b.M * ab, A->data, abytes) ||
      overlaps(dx, (size_t)b.M * ab, g, (size_t)(b.L * b.R) * ab))
    return fail(TVC_EALIAS, "dx overlaps A or g");
  if (b.total > 0 && (!ws || ws_bytes < b.total || (uintptr_t)ws % 256))
    return fail(TVC_EWORKSPACE, "workspace of " + std::to_string(b.total) + " bytes required");
  if (ws && (overlaps(ws, ws_bytes, dx, (size_t)b.M * ab)))
    return fail(TVC_EALIAS, "workspace overlaps dx");
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  const bool f8 = A->dtype == TVC_F8E4M3;
  const int accdt = A->dtype == TVC_F64 ? TVC_F64 : TVC_F32;
  if (b.kind == 1) {
    // mode 0: dx[m] = sum_r A[m, r] g[r]; slab m carries scale[m]
    return tvc_run_auto(A->dtype, A->data, b.M, b.R, 1, g, dx, 1.0, 0.0,
                        f8 ? A->slab_scale : nullptr, 1, w ? w + b.o_part : nullptr, b.part, st);
  }
  if (b.kind == 0) {
    // last mode: dx[m] = sum_l A[l, m] g[l]; row l lies in slab l / (L / n_0)
    const void* wt = g;
    if (f8) {
      float* sw = (float*)(w + b.o_w);
      hipLaunchKernelGGL(k_scale_rows, dim3(grid_(cdiv_(b.L, 256), 4)), dim3(256), 0, st,
                         (const float*)g, A->slab_scale, b.L / A->dims[0], sw, b.L);
      BX_TRY_HIP(hipGetLastError());
      wt = sw;
    }
    return tvc_run_auto(A->dtype, A->data, 1, b.L, b.M, wt, dx, 1.0, 0.0, nullptr, 1,
                        w ? w + b.o_part : nullptr, b.part, st);
  }
  // middle: P[l, m] = sum_r A[l, m, r] g[l, r] (row (l, m) uses weights g[l, :]),
  // then dx[m] = sum_l P[l, m]
  void* P = w + b.o_P;
  const bool a4 = (uintptr_t)A->data % 4 == 0, g4 = (uintptr_t)g % 4 == 0;
  TvcPlan p = plan_rows_pw(A->dtype, b.L * b.M, b.R, a4, g4, b.M);
  BX_TRY_HIP(run_rows_pw(A->dtype, A->data, b.L * b.M, b.R, g, b.M, b.R, P,
                         f8 ? A->slab_scale : nullptr, b.M * (b.L / A->dims[0]), p, w + b.o_part, st));
  void* ones = w + b.o_ones;
  if (accdt == TVC_F64)
    hipLaunchKernelGGL((k_fill<double>), dim3(grid_(cdiv_(b.L, 256), 4)), dim3(256), 0, st,
                       (double*)ones, b.L, 1.0);
  else
    hipLaunchKernelGGL((k_fill<float>), dim3(grid_(cdiv_(b.L, 256), 4)), dim3(256), 0, st,
                       (float*)ones, b.L, 1.0f);
  BX_TRY_HIP(hipGetLastError());
  return tvc_run_auto(accdt, P, 1, b.L, b.M, ones, dx, 1.0, 0.0, nullptr, 1, w + b.o_part, b.part, st);
}

int32_t tvc_backward_A(int32_t order, const int64_t* dims, int32_t dtype, int32_t mode,
                       const void* g, const void* x, void* dA, double alpha, double beta,
                       void* stream) {
  if (order < 1 || order > TVC_MAX_ORDER || !dims) return fail(TVC_EINVAL, "bad order or dims");
  if (dtype != TVC_F32 && dtype != TVC_F64) return fail(TVC_EDTYPE, "dA must be TVC_F32 or TVC_F64");
  if (mode < 0 || mode >= order) return fail(TVC_EINVAL, "mode outside [0, order)");
  if (!g || !x || !dA) return fail(TVC_EINVAL, "NULL pointer");
  tvc_tensor t{};
  t.order = order;
  t.dtype = dtype;
  for (int i = 0; i < order; ++i) t.dims[i] = dims[i];
  t.data = dA;
  tvc_status s = check_tensor(&t, "dA");
  if (s != TVC_OK) return s;
  i64 L, M, R;
  mode_view(&t, mode, &L, &M, &R);
  const size_t ab = acc_bytes(dtype);
  const i64 N = L * M * R;
  if ((uintptr_t)g % ab || (uintptr_t)x % ab) return fail(TVC_EINVAL, "g or x misaligned");
  if (overlaps(dA, (size_t)N * ab, g, (size_t)(L * R) * ab) || overlaps(dA, (size_t)N * ab, x, (size_t)M * ab))
    return fail(TVC_EALIAS, "dA overlaps g or x");
  hipStream_t st = (hipStream_t)stream;
  // rows of the [L*M][R] view, or of the [L][M] view when R == 1
  const bool byrow = R == 1;
  const i64 rows = byrow ? L : L * M;
  const i64 n = byrow ? M : R;
  const i64 eu = (i64)(16 / ab);
  const bool vec = n >= eu;
  const i64 upr = vec ? n / eu : n;
  const int tail = vec ? (int)(n % eu) : 0;
  const i64 nu = upr + (tail > 0 ? 1 : 0);
  int glog = 0;
  while (((i64)1 << glog) < nu && glog < 6) ++glog;
  const i64 chunk = nu > kWave ? std::min<i64>(nu, 16 * kWave) : nu;
  const i64 nch = cdiv_(nu, chunk);
  const i64 cbk = std::min<i64>(nch, 16);
  const i64 tasks = cdiv_(nch, cbk) * cdiv_(rows, kWave >> glog) * cbk;
  const dim3 grd(grid_(cdiv_(tasks, kBlock / kWave))), blk(kBlock);
  const bool b = beta != 0.0;
#define OUTER(T)                                                                                   \
  do {                                                                                             \
    const T* sp = (const T*)(byrow ? g : x); const T* vp = (const T*)(byrow ? x : g);              \
    const i64 smod = byrow ? L : M, vdiv = byrow ? L : M;                                          \
    T* dp = (T*)dA;                                                                                \
    if (nch > 1) {                                                                                 \
      if (b) hipLaunchKernelGGL((k_outer_rows<T, true, true, true>), grd, blk, 0, st, sp, smod, vp, vdiv, dp, rows, n, upr, tail, glog, chunk, nch, (T)alpha, (T)beta); \
      else hipLaunchKernelGGL((k_outer_rows<T, true, false, true>), grd, blk, 0, st, sp, smod, vp, vdiv, dp, rows, n, upr, tail, glog, chunk, nch, (T)alpha, (T)beta); \
    } else if (vec) {                                                                              \
      if (b) hipLaunchKernelGGL((k_outer_rows<T, true, true, false>), grd, blk, 0, st, sp, smod, vp, vdiv, dp, rows, n, upr, tail, glog, chunk, nch, (T)alpha, (T)beta); \
      else hipLaunchKernelGGL((k_outer_rows<T, true, false, false>), grd, blk, 0, st, sp, smod, vp, vdiv, dp, rows, n, upr, tail, glog, chunk, nch, (T)alpha, (T)beta); \
    } else {                                                                                       \
      if (b) hipLaunchKernelGGL((k_outer_rows<T, false, true, false>), grd, blk, 0, st, sp, smod, vp, vdiv, dp, rows, n, upr, tail, glog, chunk, nch, (T)alpha, (T)beta); \
      else hipLaunchKernelGGL((k_outer_rows<T, false, false, false>), grd, blk, 0, st, sp, smod, vp, vdiv, dp, rows, n, upr, tail, glog, chunk, nch, (T)alpha, (T)beta); \
    }                                                                                              \
  } while (0)
  if (dtype == TVC_F64) OUTER(double);
  else OUTER(float);
#undef OUTER
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TVC_EHIP, hipGetErrorString(e));
  return TVC_OK;
}

static int rank_split(int order, const int64_t* dims, i64* rows, i64* cols) {
  // columns = the trailing modes, at least 256 of them when the tensor allows
  int h = order;
  i64 c = 1;
  while (h > 1 && c < 256) {
    --h;
    c *= dims[h];
  }
  i64 r = 1;
  for (int i = 0; i < h; ++i) r *= dims[i];
  *rows = r;
  *cols = c;
  return h;
}

size_t tvc_rank_update_workspace_bytes(int32_t order, const int64_t* dims, int32_t R) {
  if (order < 1 || order > TVC_MAX_ORDER || !dims || R < 0) return 0;
  i64 rows, cols;
  rank_split(order, dims, &rows, &cols);
  // sized for double factors (float needs half)
  return align256((size_t)R * rows * 8) + align256((size_t)R * cols * 8);
}

}  // extern "C"

template <typename T>
static tvc_status rank_update_t(int order, const int64_t* dims, const T* A, double alpha, int R,
                                const double* factors, const double* coef, T* D, void* ws,
                                hipStream_t st) {
  i64 rows, cols;
  const int h = rank_split(order, dims, &rows, &cols);
  FactorArgs fa{};
  fa.h = h;
  fa.d = order;
  fa.nsum = 0;
  for (int i = 0; i < order; ++i) {
    fa.dims[i] = dims[i];
    fa.offs[i] = fa.nsum;
    fa.nsum += dims[i];
  }
  T* P = (T*)ws;
  T* Q = (T*)((char*)ws + align256((size_t)R * rows * 8));
  if (R > 0) {
    hipLaunchKernelGGL((k_factor_rows<T>), dim3(grid_(cdiv_(R * rows, 256), 4)), dim3(256), 0, st,
                       factors, coef, fa, R, P, rows, 0, h, 1);
    hipLaunchKernelGGL((k_factor_rows<T>), dim3(grid_(cdiv_(R * cols, 256), 4)), dim3(256), 0, st,
                       factors, coef, fa, R, Q, cols, h, order, 0);
  }
  const i64 tiles = cdiv_(rows, kTileR) * cdiv_(cols, kTileC);
  if (alpha != 0.0)
    hipLaunchKernelGGL((k_rank_update<T, true>), dim3(grid_(tiles, 4)), dim3(256), 0, st, A,
                       (T)alpha, (const T*)P, (const T*)Q, R, rows, cols, D);
  else
    hipLaunchKernelGGL((k_rank_update<T, false>), dim3(grid_(tiles, 4)), dim3(256), 0, st, A,
                       (T)0, (const T*)P, (const T*)Q, R, rows, cols, D);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TVC_EHIP, hipGetErrorString(e));
  return TVC_OK;
}

extern "C" {

int32_t tvc_rank_update(int32_t order, const int64_t* dims, int32_t dtype, const void* A,
                        double alpha, int32_t R, const double* factors, const double* coef,
                        void* D, void* ws, size_t ws_bytes, void* stream) {
  if (order < 1 || order > TVC_MAX_ORDER || !dims) return fail(TVC_EINVAL, "bad order or dims");
  if (dtype != TVC_F32 && dtype != TVC_F64) return fail(TVC_EDTYPE, "dtype must be TVC_F32 or TVC_F64");
  if (R < 0 || R > 4096) return fail(TVC_EINVAL, "R outside [0, 4096]");
  if (!D || (R > 0 && (!factors || !coef)) || (alpha != 0.0 && !A))
    return fail(TVC_EINVAL, "NULL pointer");
  tvc_tensor t{};
  t.order = order;
  t.dtype = dtype;
  for (int i = 0; i < order; ++i) t.dims[i] = dims[i];
  t.data = D;
  tvc_status s = check_tensor(&t, "D");
  if (s != TVC_OK) return s;
  const size_t need = tvc_rank_update_workspace_bytes(order, dims, R);
  if (need > 0 && (!ws || ws_bytes < need || (uintptr_t)ws % 256))
    return fail(TVC_EWORKSPACE, "workspace of " + std::to_string(need) + " bytes required");
  const size_t nb = (size_t)numel(&t) * elem_bytes(dtype);
  if (A && A != D && overlaps(A, nb, D, nb)) return fail(TVC_EALIAS, "A and D overlap partially");
  if (ws && (overlaps(ws, ws_bytes, D, nb) || (A && overlaps(ws, ws_bytes, A, nb))))
    return fail(TVC_EALIAS, "workspace overlaps A or D");
  hipStream_t st = (hipStream_t)stream;
  if (dtype == TVC_F64)
    return rank_update_t<double>(order, dims, (const double*)A, alpha, R, factors, coef, (double*)D,
                                 ws, st);
  return rank_update_t<float>(order, dims, (const float*)A, alpha, R, factors, coef, (float*)D, ws,
                              st);
}

}  // extern "C"
