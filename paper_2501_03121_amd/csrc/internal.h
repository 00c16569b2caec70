// Internal host-side interfaces of libtvc (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/tvc.h"

namespace tvc {

typedef int64_t i64;

// Launch roles: kernels launched for tvc_contract and for the HOPM sweep are
// separate instantiations, so profiles attribute time to each.
enum Role { kRoleContract = 0, kRoleHopm = 1, kRoleRowWeights = 2 };

// Kernel families for the (left, n_k, right) = (L, M, R) view of Sec. 3.
enum Family { kRow = 0, kCol = 1, kSlab = 2, kStage = 3 };

// Launch parameters chosen by plan_tvc (or forced by tvc_set_tuning).
struct TvcPlan {
  int family = kRow;
  bool vec = false;      // 16-byte units (dword-aligned rows)
  int tail = 0;          // vector path: elements after the last full unit of a row
  bool lng = true;       // kRow: a wave per row (true) or several rows per wave
  int glog = 0;          // log2 lanes per row (short rows / slabs)
  int rb = 1;            // kRow long: rows sharing one weight load
  int splitm = 1;        // kCol: wave groups splitting the contracted extent
  int nsplit = 1;        // split of the contracted extent across tasks
  i64 chunk = 0;         // units (kRow) or rows (kCol/kSlab) per split
  i64 upr = 0;           // units per row
  i64 tasks = 0;         // independent work items (waves or workgroups)
  int grid = 1;          // workgroups launched
  size_t part_bytes = 0; // partial-sum scratch (nsplit > 1)
  i64 sb = 0;            // kStage: slabs per LDS block
  int stage_vb = 0;      // kStage: 16 = 16-byte LDS reads, 0 = one element per read
  bool win = false;      // outputs written through an LDS window in bursts
  int wv = 4;            // waves per workgroup of the column-strip and windowed slab kernels
  bool strips = false;   // kCol: column strips, a wave per strip (k_colw)
  int cpt = 1;           // kCol strips: column units per lane
  bool mrot = false;     // kCol strips with the window: workgroup w starts at row w mod M
};

struct Tuning {
  int strip_rows = 0;      // HOPM pass 1 as strips with register weights: 1 on, -1 off, 0 built-in rule
  int blocks_per_cu[4] = {0, 0, 0, 0};
  bool stage_off = false;  // never pick the LDS-staged family
  bool win_off = false;    // never write outputs through an LDS window
  bool strips_off = false; // never use the column-strip kernel
  int split_m = 0;
};
Tuning& tuning();

// Elements' storage size, accumulation size.
size_t elem_bytes(int dtype);
size_t acc_bytes(int dtype);
int device_cus();

// a4 / w4: A / the weights start on a 4-byte boundary; a16: A starts on a
// 16-byte boundary (the LDS-staged family needs it; false is always safe
// for sizing workspaces, which the staged family never needs).
TvcPlan plan_tvc(int dtype, i64 L, i64 M, i64 R, bool a4, bool w4, bool a16 = false);

// y[l, r] = alpha * oscale[l / odiv] * sum_m A[l, m, r] * w[m] + beta * y[l, r]
// w, y, part: accumulation type of `dtype` (double for TVC_F64, else float).
// oscale may be NULL.  part: plan.part_bytes of scratch (may be NULL if 0).
hipError_t run_tvc(int dtype, const void* A, i64 L, i64 M, i64 R, const void* w,
                   void* y, double alpha, double beta, const float* oscale,
                   i64 odiv, const TvcPlan& p, void* part, hipStream_t st,
                   int role = kRoleContract);

// Rows whose weight vector depends on the row (row i uses
// w + (i / wdiv) * wstride): y[i] = oscale[i / odiv] * sum_m A[i, m] * w_i[m].
// wdiv: rows i and j share weights when i / wdiv == j / wdiv; the plan only
// puts rows that share weights in one wave.
TvcPlan plan_rows_pw(int dtype, i64 L, i64 M, bool a4, bool w4, i64 wdiv);
hipError_t run_rows_pw(int dtype, const void* A, i64 L, i64 M, const void* w, i64 wdiv,
                       i64 wstride, void* y, const float* oscale, i64 odiv, const TvcPlan& p,
                       void* part, hipStream_t st);

// Convenience: plan + run with a workspace (error if too small).
tvc_status tvc_run_auto(int dtype, const void* A, i64 L, i64 M, i64 R,
                        const void* w, void* y, double alpha, double beta,
                        const float* oscale, i64 odiv, void* ws, size_t ws_bytes,
                        hipStream_t st, int role = kRoleContract);

// One pass over A viewed as P rows of R elements giving both
//   m[p] = oscale[p / odiv] * sum_c A[p, c] w[c]   and   z[c] = sum_p u[p] A[p, c]
// (the two contractions of a Jacobi HOPM sweep).  w, u, m, z: accumulation
// type of `dtype`; part: plan.part_bytes of scratch.
struct DualPlan {
  bool cols = true;          // false: rows only (m), z is not formed
  bool vec = false;          // 16-byte units (dword-aligned rows of at least one unit)
  i64 ucount = 0;            // column units per row
  i64 nstrips = 1;           // strips of 64 * CPT units (row partials when > 1)
  i64 nchunks = 1;           // chunks of rows (column partials when > 1)
  i64 rows_per_chunk = 0;
  size_t m_part_bytes = 0, z_part_bytes = 0, part_bytes = 0;
  int grid = 1;
};
DualPlan plan_dual(int dtype, i64 P, i64 R, bool a4, bool cols = true);
hipError_t run_dual(int dtype, const void* A, i64 P, i64 R, const void* w, const void* u, void* m,
                    void* z, const float* oscale, i64 odiv, const DualPlan& p, void* part,
                    hipStream_t st);

// Round up to 256 bytes (workspace carving).
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Thread-local error message.
void set_error(const std::string& msg);
tvc_status fail(tvc_status s, const std::string& msg);

// Validation shared by the entry points.
tvc_status check_tensor(const tvc_tensor* A, const char* what);
i64 numel(const tvc_tensor* A);
void mode_view(const tvc_tensor* A, int mode, i64* L, i64* M, i64* R);
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes);

}  // namespace tvc
