// C entry points of libtvc: argument validation, the (L, M, R) view of
// Sec. 3, workspace accounting and error reporting.  Kernels live in the
// other translation units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "internal.h"

namespace tvc {

namespace {
thread_local std::string g_err;
std::mutex g_cu_mu;
std::vector<int> g_cus;  // per device
}  // namespace

// Scratch of tvc_contract_noalloc: a fixed device array (each device the
// library runs on holds its own copy until the process ends).  Host code
// never passes the array's name to a kernel or a copy (on the host it only
// stands for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device: address of `scratch` there

tvc_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(TVC_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TVC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TVC_OK;
}
}  // namespace

Tuning& tuning() {
  static Tuning t;
  return t;
}

void set_error(const std::string& msg) { g_err = msg; }

tvc_status fail(tvc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

size_t elem_bytes(int dtype) {
  switch (dtype) {
    case TVC_F64: return 8;
    case TVC_F32: return 4;
    case TVC_F16:
    case TVC_BF16: return 2;
    case TVC_F8E4M3: return 1;
    default: return 0;
  }
}

size_t acc_bytes(int dtype) { return dtype == TVC_F64 ? 8 : 4; }

int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lk(g_cu_mu);
  if ((int)g_cus.size() <= dev) g_cus.resize(dev + 1, 0);
  if (g_cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    g_cus[dev] = n;
  }
  return g_cus[dev];
}

i64 numel(const tvc_tensor* A) {
  i64 n = 1;
  for (int i = 0; i < A->order; ++i) n *= A->dims[i];
  return n;
}

tvc_status check_tensor(const tvc_tensor* A, const char* what) {
  if (!A) return fail(TVC_EINVAL, std::string(what) + " is NULL");
  if (A->order < 1 || A->order > TVC_MAX_ORDER)
    return fail(TVC_EINVAL, std::string(what) + ": order " + std::to_string(A->order) +
                                " outside [1, 16]");
  if (elem_bytes(A->dtype) == 0)
    return fail(TVC_EDTYPE, std::string(what) + ": unknown dtype " + std::to_string(A->dtype));
  i64 n = 1;
  for (int i = 0; i < A->order; ++i) {
    const i64 d = A->dims[i];
    if (d < 1) return fail(TVC_EINVAL, std::string(what) + ": dims[" + std::to_string(i) + "] < 1");
    if (n > INT64_MAX / d / 8) return fail(TVC_EINVAL, std::string(what) + ": size overflows int64");
    n *= d;
  }
  if (!A->data) return fail(TVC_EINVAL, std::string(what) + ": data is NULL");
  if ((uintptr_t)A->data % elem_bytes(A->dtype) != 0)
    return fail(TVC_EINVAL, std::string(what) + ": data not aligned to the element size");
  if (A->dtype == TVC_F8E4M3) {
    if (!A->slab_scale) return fail(TVC_EDTYPE, std::string(what) + ": F8E4M3 needs slab_scale");
    if ((uintptr_t)A->slab_scale % 4 != 0)
      return fail(TVC_EINVAL, std::string(what) + ": slab_scale misaligned");
  }
  return TVC_OK;
}

void mode_view(const tvc_tensor* A, int mode, i64* L, i64* M, i64* R) {
  i64 l = 1, r = 1;
  for (int i = 0; i < mode; ++i) l *= A->dims[i];
  for (int i = mode + 1; i < A->order; ++i) r *= A->dims[i];
  *L = l;
  *M = A->dims[mode];
  *R = r;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + abytes;
  const uintptr_t b0 = (uintptr_t)b, b1 = b0 + bbytes;
  return a0 < b1 && b0 < a1;
}

// w[m] = x[m] * scale[m]: folds the mode-0 slab scale of an E4M3 tensor into
// the weights when the contracted mode is mode 0.
__global__ void k_scale_weights(const float* x, const float* scale, float* w, i64 n) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    w[i] = x[i] * scale[i];
}

}  // namespace tvc

using namespace tvc;

extern "C" {

const char* tvc_status_string(int32_t s) {
  switch (s) {
    case TVC_OK: return "TVC_OK";
    case TVC_EINVAL: return "TVC_EINVAL";
    case TVC_EDTYPE: return "TVC_EDTYPE";
    case TVC_EALIAS: return "TVC_EALIAS";
    case TVC_EWORKSPACE: return "TVC_EWORKSPACE";
    case TVC_EHIP: return "TVC_EHIP";
    case TVC_EDEGENERATE: return "TVC_EDEGENERATE";
    case TVC_ENOTCONVERGED: return "TVC_ENOTCONVERGED";
    default: return "TVC_UNKNOWN";
  }
}

const char* tvc_last_error(void) { return g_err.c_str(); }

int32_t tvc_version(void) { return 100; }

static size_t contract_ws(const tvc_tensor* A, int32_t mode, i64 L, i64 M, i64 R) {
  size_t b = 0;
  if (A->dtype == TVC_F8E4M3 && mode == 0) b += align256((size_t)M * 4);
  const bool a4 = ((uintptr_t)A->data % 4) == 0;
  // weights live in the workspace (aligned) for E4M3 mode 0; otherwise the
  // caller's x decides the vector path, which never needs more scratch.
  TvcPlan p = plan_tvc(A->dtype, L, M, R, a4, true);
  TvcPlan q = plan_tvc(A->dtype, L, M, R, a4, false);
  b += std::max(p.part_bytes, q.part_bytes);
  return b;
}

size_t tvc_contract_workspace_bytes(const tvc_tensor* A, int32_t mode) {
  if (check_tensor(A, "A") != TVC_OK) return 0;
  if (mode < 0 || mode >= A->order) return 0;
  i64 L, M, R;
  mode_view(A, mode, &L, &M, &R);
  return contract_ws(A, mode, L, M, R);
}

int32_t tvc_contract(const tvc_tensor* A, int32_t mode, const void* x, void* y, double alpha,
                     double beta, void* ws, size_t ws_bytes, void* stream) {
  tvc_status s = check_tensor(A, "A");
  if (s != TVC_OK) return s;
  if (mode < 0 || mode >= A->order)
    return fail(TVC_EINVAL, "mode " + std::to_string(mode) + " outside [0, order)");
  if (!x || !y) return fail(TVC_EINVAL, "x or y is NULL");
  const size_t ab = acc_bytes(A->dtype);
  if ((uintptr_t)x % ab != 0 || (uintptr_t)y % ab != 0)
    return fail(TVC_EINVAL, "x or y not aligned to its element size");
  i64 L, M, R;
  mode_view(A, mode, &L, &M, &R);
  const size_t abytes = (size_t)numel(A) * elem_bytes(A->dtype);
  const size_t ybytes = (size_t)(L * R) * ab;
  const size_t xbytes = (size_t)M * ab;
  if (overlaps(y, ybytes, A->data, abytes) || overlaps(y, ybytes, x, xbytes))
    return fail(TVC_EALIAS, "y overlaps A or x");
  const size_t need = contract_ws(A, mode, L, M, R);
  if (need > 0 && (!ws || ws_bytes < need || (uintptr_t)ws % 256 != 0))
    return fail(TVC_EWORKSPACE, "workspace of " + std::to_string(need) +
                                    " bytes (256-byte aligned) required");
  if (ws && overlaps(ws, ws_bytes, y, ybytes))
    return fail(TVC_EALIAS, "workspace overlaps y");
  hipStream_t st = (hipStream_t)stream;
  const void* w = x;
  const float* oscale = nullptr;
  i64 odiv = 1;
  char* wsp = (char*)ws;
  size_t wsleft = ws_bytes;
  if (A->dtype == TVC_F8E4M3) {
    if (mode == 0) {
      float* sw = (float*)wsp;
      const int g = (int)std::min<i64>((M + 255) / 256, 1024);
      hipLaunchKernelGGL(k_scale_weights, dim3(g), dim3(256), 0, st, (const float*)x,
                         A->slab_scale, sw, M);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return fail(TVC_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
      w = sw;
      const size_t used = align256((size_t)M * 4);
      wsp += used;
      wsleft -= used;
    } else {
      oscale = A->slab_scale;
      odiv = L / A->dims[0];
    }
  }
  return tvc_run_auto(A->dtype, A->data, L, M, R, w, y, alpha, beta, oscale, odiv,
                      wsleft ? (void*)wsp : nullptr, wsleft, st);
}

size_t tvc_contract_noalloc_max_scratch(void) { return kNoAllocScratchBytes; }

int32_t tvc_contract_noalloc(const tvc_tensor* A, int32_t mode, const void* x, void* y,
                             double alpha, double beta, void* stream) {
  tvc_status s = check_tensor(A, "A");
  if (s != TVC_OK) return s;
  if (mode < 0 || mode >= A->order)
    return fail(TVC_EINVAL, "mode " + std::to_string(mode) + " outside [0, order)");
  i64 L, M, R;
  mode_view(A, mode, &L, &M, &R);
  const size_t need = contract_ws(A, mode, L, M, R);
  if (need > kNoAllocScratchBytes)
    return fail(TVC_EWORKSPACE, "this contraction needs " + std::to_string(need) +
                                    " bytes of scratch, above the " +
                                    std::to_string(kNoAllocScratchBytes) +
                                    " bytes tvc_contract_noalloc holds; use tvc_contract");
  void* p = nullptr;
  if (need > 0) {
    s = scratch_address(&p);
    if (s != TVC_OK) return s;
  }
  // the kernels write every scratch value they read (split partials are
  // stored whole before the finalize pass adds them): nothing to clear
  return tvc_contract(A, mode, x, y, alpha, beta, p, need > 0 ? kNoAllocScratchBytes : 0, stream);
}

int32_t tvc_set_tuning(int32_t family, int32_t blocks_per_cu, int32_t split_m) {
  if (family == 4) {   // HOPM pass 1 as register-weight strips
    tuning().strip_rows = blocks_per_cu > 0 ? 1 : (blocks_per_cu < 0 ? -1 : 0);
    return TVC_OK;
  }
  if (family < 0 || family > 3) return fail(TVC_EINVAL, "family outside [0, 4]");
  if (family == kStage) tuning().stage_off = blocks_per_cu < 0;
  if (family == kCol) tuning().win_off = tuning().strips_off = split_m < 0;
  if (split_m > 0 && split_m != 1 && split_m != 2 && split_m != 4)
    return fail(TVC_EINVAL, "split_m must be 1, 2 or 4");
  if (blocks_per_cu > 64) return fail(TVC_EINVAL, "blocks_per_cu above 64");
  tuning().blocks_per_cu[family] = blocks_per_cu > 0 ? blocks_per_cu : 0;
  if (family == kCol) tuning().split_m = split_m > 0 ? split_m : 0;
  return TVC_OK;
}

int32_t tvc_contract_plan(const tvc_tensor* A, int32_t mode, int32_t* info, int32_t n) {
  tvc_status s = check_tensor(A, "A");
  if (s != TVC_OK) return s;
  if (mode < 0 || mode >= A->order)
    return fail(TVC_EINVAL, "mode " + std::to_string(mode) + " outside [0, order)");
  if (!info || n < 0) return fail(TVC_EINVAL, "info is NULL");
  i64 L, M, R;
  mode_view(A, mode, &L, &M, &R);
  const bool a4 = ((uintptr_t)A->data % 4) == 0;
  const bool a16 = ((uintptr_t)A->data % 16) == 0;
  TvcPlan p = plan_tvc(A->dtype, L, M, R, a4, true, a16);
  const int32_t v[12] = {p.family, p.vec ? 1 : 0, p.splitm, p.nsplit, p.grid,
                         (p.family == kCol || (p.family == kRow && p.lng)) ? 0 : (1 << p.glog),
                         p.tail, (int32_t)std::min<i64>(p.upr, INT32_MAX), p.win ? 1 : 0,
                         (p.family == kCol && p.strips) ? p.cpt : 0, p.mrot ? 1 : 0,
                         p.family == kStage ? (int32_t)p.sb : 0};
  for (int i = 0; i < n && i < 12; ++i) info[i] = v[i];
  return TVC_OK;
}

}  // extern "C"
