// One pass over A that gives the two contractions a Jacobi HOPM sweep needs
// from the same vectors.  A is viewed as P rows of R contiguous elements
// (P = n_0 n_1 and R = n_2 ... n_{d-1} for order d >= 3; P = n_0, R = n_1 for
// a matrix), with weights w (R values) and u (P values):
//   m[p] = oscale[p / odiv] * sum_c A[p, c] w[c]      rows against w
//   z[c] = sum_p u[p] A[p, c]                          columns against u
// Each element of A is loaded once and used in two FMAs, so the pass is
// HBM-bound like a single contraction (4 flops per element).
//
// Work split: a wave owns a strip of 64 * CPT column units (16-byte vectors,
// or single elements on the scalar path) of a chunk of consecutive rows.  Its
// lanes keep the strip's weights and column sums in registers while they
// stream down the rows (each wave load is 1 KB contiguous); a row's partial
// dot is summed across the wave and stored per strip.  Several strips add
// their row partials, several chunks their column partials, in fixed order
// (finalize_sums), so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace tvc {

namespace {

constexpr int kDualWaves = 4;            // waves per 256-thread workgroup
constexpr i64 kDualWavesPerCu = 16;      // resident waves per CU of a full grid
constexpr i64 kDualTaskBytes = 32768;    // a task's fixed cost, in bytes of its strip's rows
constexpr i64 kDualMinRows = 16;         // rows per chunk, at least

template <typename Acc>
struct DualArgs {
  const void* A;
  const Acc* w;        // R weights of the rows
  const Acc* u;        // P weights of the columns
  Acc* m;              // P row results (nstrips == 1) or nstrips * P partials
  Acc* z;              // R column results (nchunks == 1) or nchunks * R partials
  const float* oscale; // optional row scale (applied when nstrips == 1)
  i64 odiv;
  i64 P, R;
  i64 ucount;          // column units per row
  i64 nstrips, nchunks, rows_per_chunk;
};

// A lane's unit i of strip s: unit index, first column it loads (the last
// unit of a ragged row is moved back to end at the row end), first column it
// owns.  Lanes past the row end load the last unit and own nothing.
template <int EU>
__device__ __forceinline__ void unit_cols(i64 un, i64 ucount, i64 R, i64& cs, i64& own) {
  if (un < ucount) {
    own = un * EU;
    cs = own < R - EU ? own : R - EU;
  } else {
    own = R;
    cs = R - EU;
  }
}

// COLS = false: rows only (m; no column sums), the row contraction of a
// Gauss-Seidel sweep's first pass with the strip's weights kept in registers.
template <int DT, bool VEC, int CPT, int RB, bool COLS>
__global__ __launch_bounds__(kDualWaves * kWave) void k_dual(DualArgs<typename St<DT>::Acc> a) {
  typedef Unit<DT, VEC> U;
  typedef typename St<DT>::Acc Acc;
  constexpr int EU = U::EU;
  const int lane = lane_id();
  const i64 wave = (i64)blockIdx.x * kDualWaves + threadIdx.x / kWave;
  const i64 nwaves = (i64)gridDim.x * kDualWaves;
  const i64 ntasks = a.nstrips * a.nchunks;
  for (i64 t = wave; t < ntasks; t += nwaves) {
    i64 q, s;
    divmod(t, a.nstrips, q, s);
    const i64 p0 = q * a.rows_per_chunk;
    const i64 p1 = p0 + a.rows_per_chunk < a.P ? p0 + a.rows_per_chunk : a.P;
    i64 cs[CPT], own[CPT];
    Acc wr[CPT][EU], col[CPT][EU];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const i64 un = s * (kWave * CPT) + (i64)i * kWave + lane;
      unit_cols<EU>(un, a.ucount, a.R, cs[i], own[i]);
#pragma unroll
      for (int e = 0; e < EU; ++e) {
        wr[i][e] = (cs[i] + e >= own[i]) ? a.w[cs[i] + e] : (Acc)0;
        col[i][e] = (Acc)0;
      }
    }
    if constexpr (COLS) {
      // Both contractions: rows in blocks of 256, row r's dot kept by lane
      // (r mod 64) in slot r / 64 of the block and the block's results stored
      // together (coalesced) instead of one 4-byte store per row; the next RB
      // rows' loads are issued before the current ones are summed (same
      // sums).  Measured: Jacobi sweep 32^6 0.78 -> 0.76 ms, 1024^3 0.735 ->
      // 0.72 ms; the rows-only pass of a Gauss-Seidel sweep keeps the plain
      // loop below (E4M3 32^6 sweep 0.41 against 0.43 ms, 8^10 1.49 against
      // 1.57 with this one).
      auto load_rows = [&](i64 pb, typename U::Raw (&raw)[RB][CPT]) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const i64 p = pb + r < p1 ? pb + r : p1 - 1;   // rows past the chunk repeat its last
          const i64 base = p * a.R;
#pragma unroll
          for (int i = 0; i < CPT; ++i) raw[r][i] = U::load(a.A, base + cs[i]);
        }
      };
      typename U::Raw cur[RB][CPT];
      load_rows(p0, cur);
      for (i64 blk = p0; blk < p1; blk += 256) {
        const i64 bend = blk + 256 < p1 ? blk + 256 : p1;
        Acc keep[4] = {(Acc)0, (Acc)0, (Acc)0, (Acc)0};
        for (i64 pb = blk; pb < bend; pb += RB) {
          typename U::Raw nxt[RB][CPT];
          if (pb + RB < p1) load_rows(pb + RB, nxt);
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            if (pb + r >= bend) break;   // wave-uniform
            const Acc up = COLS ? a.u[pb + r] : (Acc)0;
            Acc dot = (Acc)0;
#pragma unroll
            for (int i = 0; i < CPT; ++i) {
              Acc v[EU];
              U::unpack(cur[r][i], v);
#pragma unroll
              for (int e = 0; e < EU; ++e) {
                dot = fma(v[e], wr[i][e], dot);
                if constexpr (COLS) col[i][e] = fma(up, v[e], col[i][e]);
              }
            }
            dot = group_sum(dot, 6);
            const int rl = (int)(pb + r - blk);
#pragma unroll
            for (int sl = 0; sl < 4; ++sl)
              if (sl == (rl >> 6) && lane == (rl & 63)) keep[sl] = dot;
          }
#pragma unroll
          for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < CPT; ++i) cur[r][i] = nxt[r][i];
        }
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
          const i64 p = blk + sl * 64 + lane;
          if (p < bend) {
            if (a.nstrips == 1) {
              Acc sc = (Acc)1;
              if (a.oscale) sc = (Acc)a.oscale[p / a.odiv];
              a.m[p] = keep[sl] * sc;
            } else {
              a.m[s * a.P + p] = keep[sl];
            }
          }
        }
      }
    } else {
      for (i64 pb = p0; pb < p1; pb += RB) {
        typename U::Raw raw[RB][CPT];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const i64 p = pb + r < p1 ? pb + r : p1 - 1;   // rows past the chunk repeat its last
          const i64 base = p * a.R;
#pragma unroll
          for (int i = 0; i < CPT; ++i) raw[r][i] = U::load(a.A, base + cs[i]);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          if (pb + r >= p1) break;   // wave-uniform
          const Acc up = COLS ? a.u[pb + r] : (Acc)0;
          Acc dot = (Acc)0;
#pragma unroll
          for (int i = 0; i < CPT; ++i) {
            Acc v[EU];
            U::unpack(raw[r][i], v);
#pragma unroll
            for (int e = 0; e < EU; ++e) {
              dot = fma(v[e], wr[i][e], dot);
              if constexpr (COLS) col[i][e] = fma(up, v[e], col[i][e]);
            }
          }
          dot = group_sum(dot, 6);
          if (lane == 0) {
            const i64 p = pb + r;
            if (a.nstrips == 1) {
              Acc sc = (Acc)1;
              if (a.oscale) sc = (Acc)a.oscale[p / a.odiv];
              a.m[p] = dot * sc;
            } else {
              a.m[s * a.P + p] = dot;
            }
          }
        }
      }
    }
    if constexpr (!COLS) continue;
    Acc* zo = a.nchunks == 1 ? a.z : a.z + q * a.R;
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      if (own[i] >= a.R) continue;
      if constexpr (VEC) {
        if (cs[i] == own[i]) {
          store_w<Acc, EU>(zo + cs[i], col[i]);
          continue;
        }
      }
#pragma unroll
      for (int e = 0; e < EU; ++e)
        if (cs[i] + e >= own[i]) zo[cs[i] + e] = col[i][e];
    }
  }
}

// Sums of K partial vectors of C values each (part[k * C + c], k < K), in a
// fixed order: out[c] = scale(c) * sum_k part[k * C + c], where scale(c) =
// oscale[c / odiv] when oscale is given.  Few partials: one thread per c.
// Many (more than kFinDirect): pass 1 sums groups of consecutive k into
// G partials per c (one thread per (c, group), consecutive threads on
// consecutive c), pass 2 sums the G group results of each c with one wave.
constexpr i64 kFinDirect = 32;
constexpr i64 kFinMaxGroups = 512;

template <typename Acc>
__global__ void k_fin_direct(const Acc* part, Acc* out, i64 C, i64 K, const float* oscale, i64 odiv) {
  for (i64 c = (i64)blockIdx.x * blockDim.x + threadIdx.x; c < C; c += (i64)gridDim.x * blockDim.x) {
    Acc s = (Acc)0;
    for (i64 k = 0; k < K; ++k) s += part[k * C + c];
    if (oscale) s *= (Acc)oscale[c / odiv];
    out[c] = s;
  }
}

template <typename Acc>
__global__ void k_fin_groups(const Acc* part, Acc* tmp, i64 C, i64 K, i64 G) {
  const i64 per = (K + G - 1) / G;
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < C * G; i += (i64)gridDim.x * blockDim.x) {
    i64 g, c;
    divmod(i, C, g, c);
    const i64 k0 = g * per, k1 = k0 + per < K ? k0 + per : K;
    Acc s = (Acc)0;
    for (i64 k = k0; k < k1; ++k) s += part[k * C + c];
    tmp[g * C + c] = s;
  }
}

template <typename Acc>
__global__ __launch_bounds__(256) void k_fin_waves(const Acc* tmp, Acc* out, i64 C, i64 G,
                                                   const float* oscale, i64 odiv) {
  const int lane = lane_id();
  for (i64 c = ((i64)blockIdx.x * blockDim.x + threadIdx.x) / kWave; c < C;
       c += (i64)gridDim.x * blockDim.x / kWave) {
    Acc s = (Acc)0;
    for (i64 g = lane; g < G; g += kWave) s += tmp[g * C + c];
    s = group_sum(s, 6);
    if (lane == 0) {
      if (oscale) s *= (Acc)oscale[c / odiv];
      out[c] = s;
    }
  }
}

i64 fin_groups(i64 K) {
  return K <= kFinDirect ? 0 : std::min<i64>((K + 7) / 8, kFinMaxGroups);
}

template <typename Acc>
hipError_t finalize_sums(const Acc* part, Acc* out, i64 C, i64 K, const float* oscale, i64 odiv,
                         Acc* tmp, hipStream_t st) {
  const int cus = device_cus();
  const i64 G = fin_groups(K);
  if (G == 0) {
    const int g = (int)std::max<i64>(1, std::min<i64>((C + 255) / 256, 4 * (i64)cus));
    hipLaunchKernelGGL((k_fin_direct<Acc>), dim3(g), dim3(256), 0, st, part, out, C, K, oscale, odiv);
    return hipGetLastError();
  }
  int g = (int)std::max<i64>(1, std::min<i64>((C * G + 255) / 256, 8 * (i64)cus));
  hipLaunchKernelGGL((k_fin_groups<Acc>), dim3(g), dim3(256), 0, st, part, tmp, C, K, G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  g = (int)std::max<i64>(1, std::min<i64>((C + 3) / 4, 8 * (i64)cus));
  hipLaunchKernelGGL((k_fin_waves<Acc>), dim3(g), dim3(256), 0, st, (const Acc*)tmp, out, C, G, oscale,
                     odiv);
  return hipGetLastError();
}

template <int DT>
constexpr int dual_cpt(bool vec) {
  return !vec ? 4 : (St<DT>::EPV <= 4 ? 4 : (St<DT>::EPV == 8 ? 2 : 1));
}

template <int DT, bool VEC, bool COLS>
hipError_t launch_dual(const DualArgs<typename St<DT>::Acc>& a, int grid, hipStream_t st) {
  constexpr int CPT = dual_cpt<DT>(VEC);
  constexpr int RB = 8 / CPT;
  hipLaunchKernelGGL((k_dual<DT, VEC, CPT, RB, COLS>), dim3(grid), dim3(kDualWaves * kWave), 0, st, a);
  return hipGetLastError();
}

template <int DT>
hipError_t run_dual_dt(const void* A, i64 P, i64 R, const void* w, const void* u, void* m, void* z,
                       const float* oscale, i64 odiv, const DualPlan& p, void* part, hipStream_t st) {
  typedef typename St<DT>::Acc Acc;
  DualArgs<Acc> a;
  a.A = A;
  a.w = (const Acc*)w;
  a.u = (const Acc*)u;
  Acc* mp = (Acc*)part;
  Acc* zp = (Acc*)((char*)part + p.m_part_bytes);
  a.m = p.nstrips > 1 ? mp : (Acc*)m;
  a.z = p.nchunks > 1 ? zp : (Acc*)z;
  a.oscale = oscale;
  a.odiv = odiv;
  a.P = P;
  a.R = R;
  a.ucount = p.ucount;
  a.nstrips = p.nstrips;
  a.nchunks = p.nchunks;
  a.rows_per_chunk = p.rows_per_chunk;
  hipError_t e;
  if (p.cols)
    e = p.vec ? launch_dual<DT, true, true>(a, p.grid, st) : launch_dual<DT, false, true>(a, p.grid, st);
  else
    e = p.vec ? launch_dual<DT, true, false>(a, p.grid, st) : launch_dual<DT, false, false>(a, p.grid, st);
  if (e != hipSuccess) return e;
  Acc* tmp = (Acc*)((char*)part + p.m_part_bytes + p.z_part_bytes);
  if (p.nstrips > 1) {
    e = finalize_sums<Acc>(mp, (Acc*)m, P, p.nstrips, oscale, odiv, tmp, st);
    if (e != hipSuccess) return e;
  }
  if (p.cols && p.nchunks > 1) e = finalize_sums<Acc>(zp, (Acc*)z, R, p.nchunks, nullptr, 1, tmp, st);
  return e;
}

}  // namespace

DualPlan plan_dual(int dtype, i64 P, i64 R, bool a4, bool cols) {
  DualPlan p;
  p.cols = cols;
  const int epv = (int)(16 / elem_bytes(dtype));
  const size_t eb = elem_bytes(dtype);
  // 16-byte units need rows at least one unit long, dword-aligned for 4-
  // and 8-byte elements (1- and 2-byte formats load at any byte address)
  p.vec = a4 && R >= epv && (((size_t)R * eb) % 4 == 0 || eb < 4);
  const int eu = p.vec ? epv : 1;
  int cpt;
  switch (dtype) {
    case TVC_F64: cpt = dual_cpt<TVC_F64>(p.vec); break;
    case TVC_F32: cpt = dual_cpt<TVC_F32>(p.vec); break;
    case TVC_F16: cpt = dual_cpt<TVC_F16>(p.vec); break;
    case TVC_BF16: cpt = dual_cpt<TVC_BF16>(p.vec); break;
    default: cpt = dual_cpt<TVC_F8E4M3>(p.vec); break;
  }
  p.ucount = (R + eu - 1) / eu;
  p.nstrips = (p.ucount + (i64)kWave * cpt - 1) / ((i64)kWave * cpt);
  const i64 max_chunks = std::max<i64>(1, (P + kDualMinRows - 1) / kDualMinRows);
  // Tasks are equal in size, so a round of them that the grid's waves do
  // not fill is paid in full: the row chunks minimise rounds x (rows per
  // task + h), h the rows of a strip that stand for a task's fixed cost
  // (its strip's weights, its row partials: kDualTaskBytes).  Measured: 63^5 pass 1, 245
  // strips, 4165 -> 3920 tasks, sweep 66 -> 73%; 13^8, 4714 strips of 169
  // rows, 1 -> 5 chunks, 68 -> 72%; Jacobi 19^7, 2419 strips, 1 -> 5
  // chunks, 50 -> 60%).  With the column sums every chunk adds R partials
  // (at most 1/32 of A's bytes, or 16 MB), and with more strips than waves they cost
  // more than the partly filled last round (Jacobi 13^8 and 10^9: 58 and
  // 63% with one chunk, 53 and 56% with 5 and 2): one chunk there.
  const i64 waves = (i64)device_cus() * kDualWavesPerCu;
  const size_t ab0 = acc_bytes(dtype);
  i64 cmax = std::min<i64>(max_chunks, 4 * ((waves + p.nstrips - 1) / p.nstrips) + 64);
  if (cols)
    cmax = std::min<i64>(cmax, std::max<i64>({(i64)1, P * (i64)eb / (32 * (i64)ab0),
                                              ((i64)16 << 20) / (R * (i64)ab0)}));
  const i64 h = std::max<i64>(1, kDualTaskBytes / ((i64)kWave * cpt * eu * (i64)eb));
  if (cols && p.nstrips > waves) cmax = 1;
  // Candidates (the planner runs on every sweep, so no long search): up to
  // 64 chunks, and the chunk counts that fill 1..16 whole rounds.
  i64 best = -1;
  p.nchunks = 1;
  auto consider = [&](i64 c) {
    if (c < 1 || c > cmax) return;
    const i64 rpc = (P + c - 1) / c;
    const i64 tasks = p.nstrips * ((P + rpc - 1) / rpc);
    const i64 t = (tasks + waves - 1) / waves * (rpc + h);
    if (best < 0 || t < best || (t == best && c < p.nchunks)) {
      best = t;
      p.nchunks = c;
    }
  };
  for (i64 c = 1; c <= 64; ++c) consider(c);
  for (i64 k = 1; k <= 16; ++k) consider(k * waves / p.nstrips);
  p.rows_per_chunk = (P + p.nchunks - 1) / p.nchunks;
  p.nchunks = (P + p.rows_per_chunk - 1) / p.rows_per_chunk;
  const size_t ab = acc_bytes(dtype);
  p.m_part_bytes = p.nstrips > 1 ? align256((size_t)(p.nstrips * P) * ab) : 0;
  p.z_part_bytes = cols && p.nchunks > 1 ? align256((size_t)(p.nchunks * R) * ab) : 0;
  // group sums of the two finalize passes (run one after the other)
  const size_t t_bytes = std::max(align256((size_t)(fin_groups(p.nstrips) * P) * ab),
                                  cols ? align256((size_t)(fin_groups(p.nchunks) * R) * ab) : 0);
  p.part_bytes = p.m_part_bytes + p.z_part_bytes + t_bytes;
  const i64 tasks = p.nstrips * p.nchunks;
  const i64 cap = waves / kDualWaves;
  p.grid = (int)std::max<i64>(1, std::min<i64>((tasks + kDualWaves - 1) / kDualWaves, cap));
  return p;
}

hipError_t run_dual(int dtype, const void* A, i64 P, i64 R, const void* w, const void* u, void* m,
                    void* z, const float* oscale, i64 odiv, const DualPlan& p, void* part,
                    hipStream_t st) {
  switch (dtype) {
    case TVC_F64: return run_dual_dt<TVC_F64>(A, P, R, w, u, m, z, oscale, odiv, p, part, st);
    case TVC_F32: return run_dual_dt<TVC_F32>(A, P, R, w, u, m, z, oscale, odiv, p, part, st);
    case TVC_F16: return run_dual_dt<TVC_F16>(A, P, R, w, u, m, z, oscale, odiv, p, part, st);
    case TVC_BF16: return run_dual_dt<TVC_BF16>(A, P, R, w, u, m, z, oscale, odiv, p, part, st);
    case TVC_F8E4M3: return run_dual_dt<TVC_F8E4M3>(A, P, R, w, u, m, z, oscale, odiv, p, part, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tvc
