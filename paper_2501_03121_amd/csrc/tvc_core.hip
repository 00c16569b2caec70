// Streaming kernels of the k-mode tensor-vector contraction on gfx950.
//
// Sec. 3 of the paper views A as the matrix A^{uv x n_k}; here the same view
// is kept three-dimensional, A[L][M][R] with L = prod_{i<k} n_i, M = n_k,
// R = prod_{i>k} n_i, and
//     y[l, r] = sum_m A[l, m, r] * w[m].
// The contraction reads every element once and does 2 flops per element, so
// it is bound by HBM bandwidth.  Each layout gets its own coalesced access:
//   kRow  (R == 1)          rows are contiguous: lanes stride along a row and
//                           a wave reduction gives y[l]; short rows put
//                           several rows in one wave with a segmented
//                           reduction.  Long rows with few of them are split
//                           along the row into chunks (partials + finalize).
//   kCol  (R large)         lanes own 16-byte column groups of one slab and
//                           stream down the M rows; wave groups of a
//                           workgroup split M and combine in LDS.
//   kSlab (R small)         a wave covers several consecutive slabs, one
//                           lane per (slab, column group), each lane
//                           streaming down its slab's rows (no reduction).
//   kStage (M*R small)      whole slabs are copied through LDS in blocks
//                           that are one contiguous stretch of A (fully
//                           coalesced whatever M and R are), and the
//                           outputs are computed from LDS.
// Splitting the contracted extent across tasks writes partial sums to a
// workspace that k_finalize reduces in a fixed order, so results do not
// depend on scheduling (no floating-point atomics).
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace tvc {

// Loads a lane keeps in flight (build-time tunables).
#ifndef TVC_UNROLL
#define TVC_UNROLL 4
#endif
#ifndef TVC_SHORT_UNROLL
#define TVC_SHORT_UNROLL 4
#endif
#ifndef TVC_SLAB_UNROLL
#define TVC_SLAB_UNROLL 8
#endif
#ifndef TVC_COL1_UNROLL
#define TVC_COL1_UNROLL 8
#endif
constexpr int kUnroll = TVC_UNROLL;             // per row: long rows, column groups
constexpr int kShortUnroll = TVC_SHORT_UNROLL;  // short rows
constexpr int kSlabUnroll = TVC_SLAB_UNROLL;    // slabs
constexpr int kCol1Unroll = TVC_COL1_UNROLL;    // column streaming with one wave group
// Short columns and slabs with the output window: WV waves per workgroup,
// each keeping 32 / WV loads in flight.  Measured on gfx950: 4 waves of 8
// loads for 32 or more rows, 8 waves of 4 loads for fewer (the per-strip
// work is then short, and more waves hide its latency).
template <int WV>
struct ColwShape {
  static constexpr int kThreads = WV * kWave;
  // 16 waves (E4M3 column strips with the window): 4 units in flight per
  // lane, 64 KB per workgroup
  static constexpr int kUnroll = WV >= 16 ? 4 : 32 / WV;
};
constexpr int kColwMaxM = 4096;  // weights staged in LDS by the column-strip kernel
// Short rows with the window: a row-group reduction per row, so more waves
// per workgroup (1024 threads) to hide its latency, 8 rows per lane per task.
#ifndef TVC_ROWSW_UNROLL
#define TVC_ROWSW_UNROLL 8
#endif
#ifndef TVC_ROWSW_WAVES
#define TVC_ROWSW_WAVES 16
#endif
constexpr int kRowswUnroll = TVC_ROWSW_UNROLL;       // rows per lane per task
constexpr int kRowswThreads = TVC_ROWSW_WAVES * 64;  // threads per workgroup

template <typename Acc>
struct RowArgs {
  const void* A; const Acc* w; Acc* y; Acc* part;
  i64 L, upr, chunk;
  int nsplit, glog;
  Acc alpha, beta;
  const float* oscale; i64 odiv;
  // kRoleRowWeights only: row i uses the weights w + (i / wdiv) * wstride
  i64 wdiv, wstride;
  i64 ld;    // row length in elements (upr full units, then tail elements)
  int tail;  // vector path: elements after the last full unit (< EU)
};

template <typename Acc>
struct ColArgs {
  const void* A; const Acc* w; Acc* y; Acc* part;
  i64 L, M, upr, R, ctiles, chunk;
  int nsplit, glog;
  Acc alpha, beta;
  const float* oscale; i64 odiv;
  int tail;  // vector path: columns after the last full unit (< EU)
  int mrot;  // k_colw with the window: rotate each workgroup's first row
};


// Work assignment of the persistent loops.  Chunked: every workgroup takes a
// contiguous range of tasks (its waves interleaved inside the range), so a
// workgroup streams a contiguous stretch of A; otherwise tasks are dealt
// round-robin over the whole grid.  Measured on gfx950: chunked ranges help
// the long-row kernel (about 7% on 4 KB rows), round-robin dealing is 3-6%
// better for the column, slab and short-row kernels; the kernels with the
// LDS output window need contiguous ranges (block_range below).
struct TaskRange {
  i64 begin, end, step;
};

template <bool CHUNKED>
__device__ __forceinline__ TaskRange wave_tasks(i64 ntasks) {
  constexpr int wpb = kBlock / kWave;
  // the wave index is uniform across the wave; saying so keeps task indices
  // and row bases in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if constexpr (CHUNKED) {
    const i64 per = (ntasks + gridDim.x - 1) / gridDim.x;
    const i64 b = (i64)blockIdx.x * per;
    return TaskRange{b + w, min(ntasks, b + per), (i64)wpb};
  } else {
    return TaskRange{(i64)blockIdx.x * wpb + w, ntasks, (i64)gridDim.x * wpb};
  }
}

__device__ __forceinline__ TaskRange block_tasks(i64 ntasks) {
  return TaskRange{(i64)blockIdx.x, ntasks, (i64)gridDim.x};
}

// A contiguous range of tasks per workgroup.
__device__ __forceinline__ TaskRange block_range(i64 ntasks) {
  const i64 per = (ntasks + gridDim.x - 1) / gridDim.x;
  const i64 b = (i64)blockIdx.x * per;
  return TaskRange{b, min(ntasks, b + per), 1};
}

// ------------------------------------------------------------ output window
// Small writes spread through a read stream cost HBM far more than their
// bytes (measured on gfx950 with 32-row columns, where y is 1/32 of A: the
// 1 KB stores of each task cut the read rate by a fifth, while the same
// outputs written in 64-128 KB bursts per workgroup cost about their bytes).
// A workgroup that produces one contiguous stretch of y in increasing order
// therefore parks finished outputs in LDS and writes them in bursts: window
// slot i holds y[org + i] (org a 16-byte boundary at or before the first
// output held), and the window is flushed when the next round of tasks'
// outputs would not fit, and at the end.  Workgroups that take equal
// ranges advance in lockstep, so their flushes fall together.
#ifndef TVC_WIN_BYTES
#define TVC_WIN_BYTES 131072
#endif
constexpr int kWinBytes = TVC_WIN_BYTES;
// longest contracted extent given a window (its weights are kept in LDS)
#ifndef TVC_WIN_MAXM
#define TVC_WIN_MAXM 256
#endif
constexpr int kWinMaxM = TVC_WIN_MAXM;
// a window holds at least one round's outputs (up to 16 waves of 64 lanes,
// each lane with 16 float outputs (columns) or 8 rows of 1 output)
static_assert(kWinBytes == 0 || kWinBytes >= 65536, "window below a round's outputs");

template <typename Acc>
struct Win {
  static constexpr int kElems = kWinBytes > 0 ? kWinBytes / (int)sizeof(Acc) : 1;
};

// Window slot 0 is y[org], the last 16-byte boundary at or before y[base],
// so whole 16-byte groups of slots land on whole 16-byte groups of y.
template <typename Acc>
__device__ __forceinline__ i64 win_origin(const Acc* y, i64 base) {
  return base - (i64)(((uintptr_t)(y + base) & 15) / sizeof(Acc));
}

// Writes y[base, end) from the window whose slot 0 is y[org]: 16-byte
// stores for the whole groups, element stores for the partial groups at
// either end.  Called by the whole workgroup.
template <typename Acc, int NT = kBlock>
__device__ __forceinline__ void win_flush(Acc* y, const Acc* win, i64 org, i64 base, i64 end) {
  constexpr int V = 16 / (int)sizeof(Acc);
  __syncthreads();
  const int lo = (int)(base - org), hi = (int)(end - org);
  const int g0 = (lo + V - 1) / V, g1 = hi / V;
  Acc* dst = y + org;
  if (g0 >= g1) {
    for (int i = lo + threadIdx.x; i < hi; i += NT) dst[i] = win[i];
  } else {
    const int head = g0 * V - lo, tail = hi - g1 * V;
    if ((int)threadIdx.x < head) dst[lo + threadIdx.x] = win[lo + threadIdx.x];
    if ((int)threadIdx.x >= NT - tail) {
      const int i = g1 * V + (threadIdx.x - (NT - tail));
      dst[i] = win[i];
    }
    for (int g = g0 + threadIdx.x; g < g1; g += NT)
      __builtin_nontemporal_store(*(const u32x4*)(win + g * V), (u32x4*)(dst + g * V));
  }
  __syncthreads();
}

// EU consecutive values to dst; a ragged last unit stores only its elements
// from..EU-1 (the ones not owned by the unit before it).
template <typename Acc, int EU>
__device__ __forceinline__ void store_units(Acc* dst, const Acc* v, int from) {
  if (from == 0) {
    store_w<Acc, EU>(dst, v);
  } else {
#pragma unroll
    for (int e = 0; e < EU; ++e)
      if (e >= from) dst[e] = v[e];
  }
}

template <typename Acc>
__device__ __forceinline__ Acc epilogue(Acc v, const Acc* y, i64 idx, i64 l, Acc alpha,
                                        Acc beta, const float* oscale, i64 odiv) {
  if (oscale) v *= (Acc)oscale[l / odiv];
  v *= alpha;
  if (beta != (Acc)0) v += beta * y[idx];
  return v;
}

// EU consecutive outputs at y + idx with the alpha/beta/scale epilogue.
template <typename Acc, int EU>
__device__ __forceinline__ void store_epilogue(const Acc* acc, Acc* y, i64 idx, i64 l, Acc alpha,
                                               Acc beta, const float* oscale, i64 odiv, int from) {
  Acc o[EU];
#pragma unroll
  for (int e = 0; e < EU; ++e) o[e] = epilogue(acc[e], y, idx + e, l, alpha, beta, oscale, odiv);
  store_units<Acc, EU>(y + idx, o, from);
}

// ---------------------------------------------------------------- kRow, long
// One wave per (group of RB rows, chunk of the row).  Task t -> (chunk s,
// row group g) with g fastest, so consecutive waves share a weight chunk.
// A lane keeps KU units of each of the RB rows in flight, KU * RB = 8 loads
// (the planner picks RB from the units a lane owns per row, so no load slot
// idles).  When a whole row is one pass of the wave (no split, at most 64*KU
// units), every lane sees the same units in every task, so its weights are
// loaded once, before the task loop.  Each row sums into NA partial
// accumulators (EU products fold into them in a fixed order).
template <int RB>
struct RowLongShape {
  static constexpr int KU = 8 / RB;
};

template <int DT, bool VEC, int RB, int ROLE>
__global__ __launch_bounds__(kBlock) void k_row_long(RowArgs<typename St<DT>::Acc> a) {
  typedef typename St<DT>::Acc Acc;
  typedef Unit<DT, VEC> U;
  constexpr int EU = U::EU;
  constexpr int KU = RowLongShape<RB>::KU;
  constexpr int NA = EU < 4 ? EU : 4;
  const int lane = lane_id();
  const i64 ngroups = (a.L + RB - 1) / RB;
  const i64 ntasks = ngroups * a.nsplit;
  const bool wreg = ROLE != kRoleRowWeights && a.nsplit == 1 && a.upr <= (i64)kWave * KU;
  Acc wv[KU][EU];
  if (wreg) {
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      const i64 uk = lane + (i64)k * kWave;
      if (uk < a.upr) {
        load_w<Acc, EU>(a.w, uk * EU, wv[k]);
      } else if (uk == a.upr && a.tail > 0) {
        // the ragged end as one more unit that re-reads the row's last EU
        // elements, the ones the last full unit covered weighted 0 (only
        // the preloading path below reads this unit's slot)
        load_w<Acc, EU>(a.w, a.ld - EU, wv[k]);
#pragma unroll
        for (int e = 0; e < EU; ++e)
          if (e < EU - a.tail) wv[k][e] = (Acc)0;
      } else {
#pragma unroll
        for (int e = 0; e < EU; ++e) wv[k][e] = (Acc)0;
      }
    }
  }
  const TaskRange tr = wave_tasks<true>(ntasks);
  // Rows that are one pass of the wave (weights in registers; a ragged end
  // is one more unit, if the wave has a slot for it): a wave loads its next
  // row group before summing the current one (same sums), so its
  // arithmetic (24 vector instructions per 16-byte E4M3 load) overlaps
  // loads in flight.  Measured in float32 against the plain loop: 175^4
  // mode 3 (rows of 175 values) 57 -> 71%, 979^3 mode 2 79 -> 83%, 1024^3
  // mode 2 unchanged.
  if constexpr (ROLE != kRoleRowWeights) {
    if (wreg && (a.tail == 0 || a.upr < (i64)kWave * KU)) {
      auto load_group = [&](i64 g, typename U::Raw (&raw)[KU][RB]) {
#pragma unroll
        for (int k = 0; k < KU; ++k) {
          const i64 uk = lane + (i64)k * kWave;
          // unmasked loads: a slot past the row's units reads its first
          // unit (weights 0), a row past the end re-reads the last row (not
          // stored)
          const bool full = uk < a.upr;
          const bool ok = full || (uk == a.upr && a.tail > 0);
          const i64 eo = full ? uk * EU : (ok ? a.ld - EU : 0);
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            const i64 row = g * RB + r;
            raw[k][r] = U::load(a.A, (row < a.L ? row : a.L - 1) * a.ld + eo);
          }
        }
      };
      typename U::Raw nxt[KU][RB];
      if (tr.begin < tr.end) load_group(tr.begin, nxt);
      for (i64 t = tr.begin; t < tr.end; t += tr.step) {
        typename U::Raw raw[KU][RB];
#pragma unroll
        for (int k = 0; k < KU; ++k)
#pragma unroll
          for (int r = 0; r < RB; ++r) raw[k][r] = nxt[k][r];
        if (t + tr.step < tr.end) load_group(t + tr.step, nxt);
        Acc acc[RB][NA];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int e = 0; e < NA; ++e) acc[r][e] = (Acc)0;
#pragma unroll
        for (int k = 0; k < KU; ++k)
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            Acc v[EU];
            U::unpack(raw[k][r], v);
#pragma unroll
            for (int e = 0; e < EU; ++e) acc[r][e % NA] = fma(v[e], wv[k][e], acc[r][e % NA]);
          }
        // the butterfly reduction and store of the general path below
        Acc v[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          v[r] = (Acc)0;
#pragma unroll
          for (int e = 0; e < NA; ++e) v[r] += acc[r][e];
        }
        int rsel = 0;
#pragma unroll
        for (int h = RB / 2, off = kWave / 2; h >= 1; h /= 2, off /= 2) {
          const bool up = (lane & off) != 0;
#pragma unroll
          for (int i = 0; i < h; ++i) {
            const Acc keep = up ? v[i + h] : v[i];
            const Acc send = up ? v[i] : v[i + h];
            v[i] = keep + shfl_xor(send, off);
          }
          rsel += up ? h : 0;
        }
        Acc s_ = v[0];
#pragma unroll
        for (int off = kWave / (2 * RB); off >= 1; off /= 2) s_ += shfl_xor(s_, off);
        const i64 row = t * RB + rsel;
        if ((lane & (kWave / RB - 1)) == 0 && row < a.L)
          a.y[row] = epilogue(s_, a.y, row, row, a.alpha, a.beta, a.oscale, a.odiv);
      }
      return;
    }
  }
  for (i64 t = tr.begin; t < tr.end; t += tr.step) {
    i64 s, g;
    divmod(t, ngroups, s, g);
    const i64 row0 = g * RB;
    const i64 u0 = s * a.chunk;
    const i64 u1 = min(a.upr, u0 + a.chunk);
    const Acc* wr = a.w;
    if constexpr (ROLE == kRoleRowWeights) wr = a.w + (row0 / a.wdiv) * a.wstride;
    // uniform base of the chunk in each row; lanes add 32-bit byte offsets
    // (the planner keeps a chunk below 2^31 bytes)
    const char* cbase[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
      cbase[r] = (const char*)a.A + ((row0 + r) * a.ld + u0 * EU) * (i64)sizeof(typename U::T);
    Acc acc[RB][NA];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int e = 0; e < NA; ++e) acc[r][e] = (Acc)0;
    // Ragged row end (vector path): lane r < RB loads the last EU elements
    // of row r now, so that the load overlaps the stream below instead of
    // adding a round trip after it; the EU - tail elements the last full
    // unit covered are skipped when it is added.
    const bool tail_task = a.tail > 0 && s == a.nsplit - 1;
    const bool tail_lane = tail_task && lane < RB && row0 + lane < a.L;
    typename U::Raw traw = U::zero();
    if (tail_lane) traw = U::load(a.A, (row0 + lane) * a.ld + a.ld - EU);
    auto load_step = [&](i64 u, typename U::Raw (&raw)[KU][RB], Acc (&wk)[KU][EU]) {
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        const i64 uk = u + (i64)k * kWave;
        const bool ok = uk < u1;
        const uint32_t off = (uint32_t)(uk - u0) * (uint32_t)(EU * sizeof(typename U::T));
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const i64 row = row0 + r;
          raw[k][r] = (ok && row < a.L) ? U::load(cbase[r] + (uint64_t)off, 0) : U::zero();
        }
        if (!wreg) {
          if (ok) {
            load_w<Acc, EU>(wr, uk * EU, wk[k]);
          } else {
#pragma unroll
            for (int e = 0; e < EU; ++e) wk[k][e] = (Acc)0;
          }
        }
      }
    };
    auto sum_step = [&](const typename U::Raw (&raw)[KU][RB], const Acc (&wk)[KU][EU]) {
#pragma unroll
      for (int k = 0; k < KU; ++k)
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          Acc v[EU];
          U::unpack(raw[k][r], v);
#pragma unroll
          for (int e = 0; e < EU; ++e) acc[r][e % NA] = fma(v[e], wk[k][e], acc[r][e % NA]);
        }
    };
    if constexpr (sizeof(Acc) == 8 || !VEC) {
      // float64 and one-element units: the next step's loads are issued
      // before this step is summed (same sums)
      typename U::Raw cur[KU][RB];
      Acc wc[KU][EU];
      if (wreg) {
#pragma unroll
        for (int k = 0; k < KU; ++k)
#pragma unroll
          for (int e = 0; e < EU; ++e) wc[k][e] = wv[k][e];
      }
      if (u0 + lane < u1) load_step(u0 + lane, cur, wc);
      for (i64 u = u0 + lane; u < u1; u += (i64)kWave * KU) {
        typename U::Raw nxt[KU][RB];
        Acc wn[KU][EU];
        if (wreg) {
#pragma unroll
          for (int k = 0; k < KU; ++k)
#pragma unroll
            for (int e = 0; e < EU; ++e) wn[k][e] = wv[k][e];
        }
        if (u + (i64)kWave * KU < u1) load_step(u + (i64)kWave * KU, nxt, wn);
        sum_step(cur, wc);
#pragma unroll
        for (int k = 0; k < KU; ++k) {
#pragma unroll
          for (int r = 0; r < RB; ++r) cur[k][r] = nxt[k][r];
#pragma unroll
          for (int e = 0; e < EU; ++e) wc[k][e] = wn[k][e];
        }
      }
    } else {
      for (i64 u = u0 + lane; u < u1; u += (i64)kWave * KU) {
        typename U::Raw raw[KU][RB];
        load_step(u, raw, wv);
        sum_step(raw, wv);
      }
    }
    if (tail_lane) {
      const int from = EU - a.tail;
      Acc wt[EU], v[EU];
      load_w<Acc, EU>(wr, a.ld - EU, wt);
      U::unpack(traw, v);
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r == lane) {
#pragma unroll
          for (int e = 0; e < EU; ++e)
            if (e >= from) acc[r][e % NA] = fma(v[e], wt[e], acc[r][e % NA]);
        }
    }
    // Cross-lane reduction of the RB row sums as a butterfly: each of the
    // first log2(RB) exchanges hands half of a lane's rows to its partner,
    // so a lane ends with one row's partial sum (row rsel) after RB - 1
    // shuffles instead of RB * 6; the rest is a plain xor reduction among
    // the 64/RB lanes holding that row.
    Acc v[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      v[r] = (Acc)0;
#pragma unroll
      for (int e = 0; e < NA; ++e) v[r] += acc[r][e];
    }
    int rsel = 0;
#pragma unroll
    for (int h = RB / 2, off = kWave / 2; h >= 1; h /= 2, off /= 2) {
      const bool up = (lane & off) != 0;
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const Acc keep = up ? v[i + h] : v[i];
        const Acc send = up ? v[i] : v[i + h];
        v[i] = keep + shfl_xor(send, off);
      }
      rsel += up ? h : 0;
    }
    Acc s_ = v[0];
#pragma unroll
    for (int off = kWave / (2 * RB); off >= 1; off /= 2) s_ += shfl_xor(s_, off);
    const i64 row = row0 + rsel;
    if ((lane & (kWave / RB - 1)) == 0 && row < a.L) {
      if (a.nsplit > 1) a.part[s * a.L + row] = s_;
      else a.y[row] = epilogue(s_, a.y, row, row, a.alpha, a.beta, a.oscale, a.odiv);
    }
  }
}

// ---------------------------------------------------------------- kRow, short
// G = 2^glog lanes per row (G >= units per row, a ragged end counting as one
// more unit that re-reads the row's last EU elements and drops the overlap),
// 64/G rows per wave load.
template <int DT, bool VEC, int ROLE>
__global__ __launch_bounds__(kBlock) void k_row_short(RowArgs<typename St<DT>::Acc> a) {
  typedef typename St<DT>::Acc Acc;
  typedef Unit<DT, VEC> U;
  constexpr int EU = U::EU;
  const int lane = lane_id();
  const int G = 1 << a.glog;
  const int P = kWave >> a.glog;
  const int sub = lane & (G - 1);
  const int rsub = lane >> a.glog;
  const bool tl = a.tail > 0 && sub == a.upr;
  const bool active = sub < a.upr || tl;
  const i64 eo = tl ? a.ld - EU : (i64)sub * EU;
  const int from = tl ? EU - a.tail : 0;
  Acc wv[EU];
  if (active && ROLE != kRoleRowWeights) {
    load_w<Acc, EU>(a.w, eo, wv);
  } else {
#pragma unroll
    for (int e = 0; e < EU; ++e) wv[e] = (Acc)0;
  }
  const i64 per = (i64)P * kShortUnroll;
  const TaskRange tr = wave_tasks<false>((a.L + per - 1) / per);
  for (i64 t = tr.begin; t < tr.end; t += tr.step) {
    const i64 base = t * per;
    typename U::Raw raw[kShortUnroll];
#pragma unroll
    for (int k = 0; k < kShortUnroll; ++k) {
      // unmasked loads (see k_rowsw): inactive lanes read the row's first
      // unit and rows past the end the last row, with weights 0 or no store
      const i64 row = base + (i64)k * P + rsub;
      raw[k] = U::load(a.A, (row < a.L ? row : a.L - 1) * a.ld + (active ? eo : 0));
    }
#pragma unroll
    for (int k = 0; k < kShortUnroll; ++k) {
      Acc v[EU];
      U::unpack(raw[k], v);
      if (a.tail > 0) {
#pragma unroll
        for (int e = 0; e < EU; ++e) v[e] = e < from ? (Acc)0 : v[e];
      }
      if constexpr (ROLE == kRoleRowWeights) {
        const i64 row = base + (i64)k * P + rsub;
        if (active && row < a.L) load_w<Acc, EU>(a.w + (row / a.wdiv) * a.wstride, eo, wv);
      }
      Acc s_ = (Acc)0;
#pragma unroll
      for (int e = 0; e < EU; ++e) s_ = fma(v[e], wv[e], s_);
      s_ = group_sum(s_, a.glog);
      const i64 row = base + (i64)k * P + rsub;
      if (sub == 0 && row < a.L)
        a.y[row] = epilogue(s_, a.y, row, row, a.alpha, a.beta, a.oscale, a.odiv);
    }
  }
}

// ---------------------------------------------------------------- kCol
// Workgroup task = (split s, slab l, column tile ct), ct fastest.  TC threads
// along columns (one unit each), SPLITM wave groups along the rows, each
// keeping UN loads in flight; the groups combine in LDS.  A ragged row end
// is one more unit reading the last EU columns; it stores only the columns
// after the last full unit.
template <int DT, bool VEC, int SPLITM, int ROLE>
__global__ __launch_bounds__(kBlock) void k_col(ColArgs<typename St<DT>::Acc> a) {
  typedef typename St<DT>::Acc Acc;
  typedef Unit<DT, VEC> U;
  constexpr int EU = U::EU;
  constexpr int TC = kBlock / SPLITM;
  constexpr int UN = SPLITM == 1 ? kCol1Unroll : kUnroll;
  __shared__ Acc red[SPLITM > 1 ? (SPLITM - 1) * TC * EU : 1];
  const int tc = threadIdx.x % TC;
  const int grp = threadIdx.x / TC;
  const i64 ntasks = a.L * a.ctiles * a.nsplit;
  const TaskRange tr = block_tasks(ntasks);
  for (i64 t = tr.begin; t < tr.end; t += tr.step) {
    i64 ct, rest, l, s;
    divmod(t, a.ctiles, rest, ct);
    divmod(rest, a.L, s, l);
    const i64 c = ct * TC + tc;
    const bool tl = a.tail > 0 && c == a.upr;
    const bool active = c < a.upr || tl;
    const i64 eo = tl ? a.R - EU : c * EU;
    const i64 m0 = s * a.chunk;
    const i64 m1 = min(a.M, m0 + a.chunk);
    const i64 slab = l * a.M;
    Acc acc[EU];
#pragma unroll
    for (int e = 0; e < EU; ++e) acc[e] = (Acc)0;
    if constexpr (sizeof(Acc) == 8 || !VEC) {
      // float64 and one-element units: the next UN rows' loads are issued
      // before this batch is summed (same sums); loads are unmasked (a row
      // past the split reads the split's last row with weight 0, an
      // inactive lane the slab's first unit, not stored).  Measured: float64
      // 30623^2 mode 0 51 -> 75%, bf16 (rows of an odd number of elements,
      // so one element per load) 9.5 -> 25%; float32 and 16-byte bf16 units
      // gain nothing or lose (bf16 1024^3 sweep 76 -> 69%).
      auto load_batch = [&](i64 m, typename U::Raw (&raw)[UN], Acc (&wv)[UN]) {
#pragma unroll
        for (int k = 0; k < UN; ++k) {
          const i64 mk = m + (i64)k * SPLITM;
          const bool ok = mk < m1;
          raw[k] = U::load(a.A, (slab + (ok ? mk : m1 - 1)) * a.R + (active ? eo : 0));
          wv[k] = ok ? a.w[mk] : (Acc)0;
        }
      };
      typename U::Raw cur[UN];
      Acc wc[UN];
      if (m0 + grp < m1) load_batch(m0 + grp, cur, wc);
      for (i64 m = m0 + grp; m < m1; m += (i64)SPLITM * UN) {
        typename U::Raw nxt[UN];
        Acc wn[UN];
        if (m + (i64)SPLITM * UN < m1) load_batch(m + (i64)SPLITM * UN, nxt, wn);
#pragma unroll
        for (int k = 0; k < UN; ++k) {
          Acc v[EU];
          U::unpack(cur[k], v);
#pragma unroll
          for (int e = 0; e < EU; ++e) acc[e] = fma(v[e], wc[k], acc[e]);
        }
#pragma unroll
        for (int k = 0; k < UN; ++k) {
          cur[k] = nxt[k];
          wc[k] = wn[k];
        }
      }
    } else {
      for (i64 m = m0 + grp; m < m1; m += (i64)SPLITM * UN) {
        typename U::Raw raw[UN];
        Acc wv[UN];
#pragma unroll
        for (int k = 0; k < UN; ++k) {
          const i64 mk = m + (i64)k * SPLITM;
          const bool ok = mk < m1;
          raw[k] = (active && ok) ? U::load(a.A, (slab + mk) * a.R + eo) : U::zero();
          wv[k] = ok ? a.w[mk] : (Acc)0;
        }
#pragma unroll
        for (int k = 0; k < UN; ++k) {
          Acc v[EU];
          U::unpack(raw[k], v);
#pragma unroll
          for (int e = 0; e < EU; ++e) acc[e] = fma(v[e], wv[k], acc[e]);
        }
      }
    }
    if constexpr (SPLITM > 1) {
      if (grp > 0) {
#pragma unroll
        for (int e = 0; e < EU; ++e) red[((grp - 1) * TC + tc) * EU + e] = acc[e];
      }
      __syncthreads();
      if (grp == 0) {
#pragma unroll
        for (int g = 1; g < SPLITM; ++g)
#pragma unroll
          for (int e = 0; e < EU; ++e) acc[e] += red[((g - 1) * TC + tc) * EU + e];
      }
    }
    if (grp == 0 && active) {
      const i64 idx = l * a.R + eo;
      const int from = tl ? EU - a.tail : 0;
      if (a.nsplit > 1) store_units<Acc, EU>(a.part + s * (a.L * a.R) + idx, acc, from);
      else store_epilogue<Acc, EU>(acc, a.y, idx, l, a.alpha, a.beta, a.oscale, a.odiv, from);
    }
    if constexpr (SPLITM > 1) __syncthreads();
  }
}

// ------------------------------------------------------ kCol, column strips
// A wave owns a strip of CPT * 64 column units of one slab (lane owns units
// lane, lane + 64, ...) and streams all M rows of it, UN loads in flight: a
// batch is UN / CPT rows of CPT * 1 KB contiguous pieces.  No combine across
// waves, so no barrier per task; the M weights are staged in LDS once.
// Several units per lane matter when rows are a power-of-two number of MB
// apart: loads of one column unit down 8 such rows fall on few HBM channels
// (measured on gfx950, 1000 rows 4 MB apart: 5.7 TB/s with one unit per
// lane, 7.1 TB/s with four or with a 4 KB pad between rows).  A lane's units
// past the row end re-read the row's last unit and are not stored, so every
// load is unconditional.  With WIN (short M, where y is a sizeable share of
// the traffic) the strips of a workgroup's contiguous range go to its waves
// in rounds whose outputs are one stretch of y, collected in the LDS window;
// without it every output is stored as its strip finishes.

// All M rows of one strip into acc: batches of RPB rows of CPT units each,
// the last M mod RPB rows as one more batch.  With ROT the row order starts
// at row ms and wraps around (row index r + ms, less M past the end): where
// many slabs' rows are a power-of-two number of MB apart, workgroups that
// all read the same row index at once load addresses that share their low
// 20+ bits.  Measured on 32^6 float32 mode 1 (4 MB rows, 128 MB slabs): 75
// -> 84% of peak.  The same wrapped indexing costs 3-8 points where rows
// are 4 KB or 64-128 MB apart, with or without a rotation, so it is only
// compiled into the windowed kernel and taken where the planner asks.
template <class U, int RPB, int CPT, bool ROT, typename Acc>
__device__ __forceinline__ void colw_rows(const char* row0, i64 rs, const i64 (&eo)[CPT], const Acc* wl,
                                          int M, int ms, Acc (&acc)[CPT][U::EU]) {
  constexpr int EU = U::EU;
  auto rr = [&](int r) {
    if constexpr (ROT) {
      r += ms;
      return r >= M ? r - M : r;
    } else {
      return r;
    }
  };
  int m = 0;
  // The next batch's loads are issued before the current batch is summed
  // (same order of sums), so a wave's arithmetic overlaps loads in flight:
  // E4M3 (24 vector instructions per 16-byte load), float64 (32^6 modes
  // 0-3 58-73 -> 81-86%, 1024^3 modes 0-1 69-72 -> 88%) and float32 on the
  // rotated rows (32^6 mode 1: 83.5 -> 85%).  float32 and bf16 elsewhere
  // lose 2-5 points to the registers the second batch takes.
  if constexpr (EU >= 16 || sizeof(Acc) == 8 || (ROT && EU == 4)) {
    if (M >= RPB) {
      typename U::Raw cur[RPB][CPT];
#pragma unroll
      for (int q = 0; q < RPB; ++q)
#pragma unroll
        for (int j = 0; j < CPT; ++j) cur[q][j] = U::load(row0 + (i64)rr(q) * rs, eo[j]);
      for (; m + 2 * RPB <= M; m += RPB) {
        typename U::Raw nxt[RPB][CPT];
#pragma unroll
        for (int q = 0; q < RPB; ++q)
#pragma unroll
          for (int j = 0; j < CPT; ++j) nxt[q][j] = U::load(row0 + (i64)rr(m + RPB + q) * rs, eo[j]);
#pragma unroll
        for (int q = 0; q < RPB; ++q) {
          const Acc wk = wl[rr(m + q)];
#pragma unroll
          for (int j = 0; j < CPT; ++j) {
            Acc v[EU];
            U::unpack(cur[q][j], v);
#pragma unroll
            for (int e = 0; e < EU; ++e) acc[j][e] = fma(v[e], wk, acc[j][e]);
          }
        }
#pragma unroll
        for (int q = 0; q < RPB; ++q)
#pragma unroll
          for (int j = 0; j < CPT; ++j) cur[q][j] = nxt[q][j];
      }
#pragma unroll
      for (int q = 0; q < RPB; ++q) {
        const Acc wk = wl[rr(m + q)];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
          Acc v[EU];
          U::unpack(cur[q][j], v);
#pragma unroll
          for (int e = 0; e < EU; ++e) acc[j][e] = fma(v[e], wk, acc[j][e]);
        }
      }
      m += RPB;
    }
  }
  for (; m + RPB <= M; m += RPB) {
    typename U::Raw raw[RPB][CPT];
#pragma unroll
    for (int q = 0; q < RPB; ++q)
#pragma unroll
      for (int j = 0; j < CPT; ++j) raw[q][j] = U::load(row0 + (i64)rr(m + q) * rs, eo[j]);
#pragma unroll
    for (int q = 0; q < RPB; ++q) {
      const Acc wk = wl[rr(m + q)];
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        Acc v[EU];
        U::unpack(raw[q][j], v);
#pragma unroll
        for (int e = 0; e < EU; ++e) acc[j][e] = fma(v[e], wk, acc[j][e]);
      }
    }
  }
  if constexpr (RPB > 1) {
    if (m < M) {
      // the last M mod RPB rows, loads issued together (M is uniform)
      typename U::Raw raw[RPB - 1][CPT];
#pragma unroll
      for (int q = 0; q < RPB - 1; ++q)
#pragma unroll
        for (int j = 0; j < CPT; ++j)
          raw[q][j] = m + q < M ? U::load(row0 + (i64)rr(m + q) * rs, eo[j]) : U::zero();
#pragma unroll
      for (int q = 0; q < RPB - 1; ++q) {
        if (m + q < M) {
          const Acc wk = wl[rr(m + q)];
#pragma unroll
          for (int j = 0; j < CPT; ++j) {
            Acc v[EU];
            U::unpack(raw[q][j], v);
#pragma unroll
            for (int e = 0; e < EU; ++e) acc[j][e] = fma(v[e], wk, acc[j][e]);
          }
        }
      }
    }
  }
}

template <int DT, bool VEC, int ROLE, int WV, int CPT, bool WIN>
__global__ __launch_bounds__(ColwShape<WV>::kThreads) void k_colw(ColArgs<typename St<DT>::Acc> a) {
  typedef typename St<DT>::Acc Acc;
  typedef typename St<DT>::T T;
  typedef Unit<DT, VEC> U;
  constexpr int EU = U::EU;
  constexpr int NT = ColwShape<WV>::kThreads;
  constexpr int UN = ColwShape<WV>::kUnroll;
  constexpr int RPB = UN / CPT;               // rows per batch of loads
  static_assert(RPB >= 1 && RPB * CPT == UN, "CPT must divide the loads in flight");
  constexpr i64 SWU = (i64)kWave * CPT;       // column units per strip
  constexpr i64 SW = SWU * EU;                // elements of y per strip
  __shared__ __align__(16) Acc win[WIN ? Win<Acc>::kElems : 1];
  __shared__ Acc wl[WIN ? kWinMaxM : kColwMaxM];
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int M = (int)a.M;
  for (int i = threadIdx.x; i < M; i += NT) wl[i] = a.w[i];
  __syncthreads();
  const i64 rs = a.R * (i64)sizeof(T);  // row stride, bytes
  const TaskRange tr = WIN ? block_range(a.L * a.ctiles) : TaskRange{(i64)blockIdx.x * WV, a.L * a.ctiles,
                                                                     (i64)gridDim.x * WV};
  i64 org = 0, wbase = 0, wend = 0;
  for (i64 t0 = tr.begin; t0 < tr.end; t0 += (WIN ? WV : tr.step)) {
    i64 t = t0 + wv;
    if constexpr (WIN) {
      const i64 tlast = min(t0 + WV, tr.end) - 1;
      i64 l0, c0, l1, c1;
      divmod(t0, a.ctiles, l0, c0);
      divmod(tlast, a.ctiles, l1, c1);
      const i64 ys = l0 * a.R + c0 * SW;
      const i64 ye = l1 * a.R + min(a.R, (c1 + 1) * SW);
      if (t0 == tr.begin) {
        wbase = ys;
        org = win_origin(a.y, ys);
      } else if (ye - org > Win<Acc>::kElems) {
        win_flush<Acc, NT>(a.y, win, org, wbase, ys);
        wbase = ys;
        org = win_origin(a.y, ys);
      }
      wend = ye;
      if (t > tlast) continue;
    } else {
      if (t >= tr.end) break;
    }
    i64 l, ct;
    divmod(t, a.ctiles, l, ct);
    const char* row0 = (const char*)a.A + l * a.M * a.R * (i64)sizeof(T);
    i64 eo[CPT];
    bool act[CPT], tl[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const i64 c = ct * SWU + j * kWave + lane;
      tl[j] = a.tail > 0 && c == a.upr;
      act[j] = c < a.upr || tl[j];
      eo[j] = c < a.upr ? c * EU : a.R - EU;
    }
    Acc acc[CPT][EU];
#pragma unroll
    for (int j = 0; j < CPT; ++j)
#pragma unroll
      for (int e = 0; e < EU; ++e) acc[j][e] = (Acc)0;
    // With mrot, workgroup w streams rows w mod M, ..., M - 1, 0, ..., w - 1
    // (see colw_rows)
    if constexpr (WIN) {
      if (a.mrot) colw_rows<U, RPB, CPT, true>(row0, rs, eo, wl, M, (int)(blockIdx.x % (unsigned)M), acc);
      else colw_rows<U, RPB, CPT, false>(row0, rs, eo, wl, M, 0, acc);
    } else {
      colw_rows<U, RPB, CPT, false>(row0, rs, eo, wl, M, 0, acc);
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (!act[j]) continue;
      const i64 idx = l * a.R + eo[j];
      const int from = tl[j] ? EU - a.tail : 0;
      if constexpr (WIN) {
        Acc* wp = win + (idx - org);
#pragma unroll
        for (int e = 0; e < EU; ++e)
          if (e >= from) wp[e] = epilogue(acc[j][e], a.y, idx + e, l, a.alpha, a.beta, a.oscale, a.odiv);
      } else {
        store_epilogue<Acc, EU>(acc[j], a.y, idx, l, a.alpha, a.beta, a.oscale, a.odiv, from);
      }
    }
  }
  if constexpr (WIN) {
    if (tr.begin < tr.end) win_flush<Acc, NT>(a.y, win, org, wbase, wend);
  }
}

// ---------------------------------------------------------------- kSlab
// Small right extent (R <= 32 units).  A wave covers P = 64/G consecutive
// slabs: lane (q, c) = (lane / G, lane mod G) owns column unit c of slab
// l0 + q and streams down the M rows of that slab, so no cross-lane
// reduction is needed; for a fixed row a wave load reads P contiguous
// segments of G*16 bytes, one per slab.  The weight of a row is uniform
// across the wave.  A ragged row end is handled as in kCol.
template <int DT, bool VEC, int ROLE>
__global__ __launch_bounds__(kBlock) void k_slab(ColArgs<typename St<DT>::Acc> a) {
  typedef typename St<DT>::Acc Acc;
  typedef Unit<DT, VEC> U;
  constexpr int EU = U::EU;
  constexpr int UN = kSlabUnroll;
  const int lane = lane_id();
  const int G = 1 << a.glog;
  const int P = kWave >> a.glog;
  const int q = lane >> a.glog;
  const int c = lane & (G - 1);
  const i64 groups = (a.L + P - 1) / P;
  const i64 ntasks = groups * a.nsplit;
  const TaskRange tr = wave_tasks<false>(ntasks);
  for (i64 t = tr.begin; t < tr.end; t += tr.step) {
    i64 g, s;
    divmod(t, groups, s, g);
    const i64 l = g * P + q;
    const bool tl = a.tail > 0 && c == a.upr;
    const bool on = (c < a.upr || tl) && l < a.L;
    const i64 eo = tl ? a.R - EU : (i64)c * EU;
    const i64 m0 = s * a.chunk;
    const i64 m1 = min(a.M, m0 + a.chunk);
    const i64 base = l * a.M * a.R + eo;
    Acc acc[EU];
#pragma unroll
    for (int e = 0; e < EU; ++e) acc[e] = (Acc)0;
    for (i64 m = m0; m < m1; m += UN) {
      typename U::Raw raw[UN];
      Acc wv[UN];
#pragma unroll
      for (int k = 0; k < UN; ++k) {
        const i64 mk = m + k;
        const bool ok = mk < m1;
        raw[k] = (on && ok) ? U::load(a.A, base + mk * a.R) : U::zero();
        wv[k] = ok ? a.w[mk] : (Acc)0;
      }
#pragma unroll
      for (int k = 0; k < UN; ++k) {
        Acc v[EU];
        U::unpack(raw[k], v);
#pragma unroll
        for (int e = 0; e < EU; ++e) acc[e] = fma(v[e], wv[k], acc[e]);
      }
    }
    if (on) {
      const i64 idx = l * a.R + eo;
      const int from = tl ? EU - a.tail : 0;
      if (a.nsplit > 1) store_units<Acc, EU>(a.part + s * (a.L * a.R) + idx, acc, from);
      else store_epilogue<Acc, EU>(acc, a.y, idx, l, a.alpha, a.beta, a.oscale, a.odiv, from);
    }
  }
}

// ------------------------------------------------- kSlab / kRow, windowed
// The slab and short-row kernels with the LDS output window, for short
// contracted extents (the slab kernel) and short rows: a workgroup takes a
// contiguous range of wave tasks in rounds of one task per wave, whose
// outputs are one stretch of y; it is flushed as in k_colw.

// Slabs: the lane layout of k_slab; the M weights are staged in LDS and the
// row loop is unmasked.
template <int DT, bool VEC, int ROLE, int WV>
__global__ __launch_bounds__(ColwShape<WV>::kThreads) void k_slabw(ColArgs<typename St<DT>::Acc> a) {
  typedef typename St<DT>::Acc Acc;
  typedef typename St<DT>::T T;
  typedef Unit<DT, VEC> U;
  constexpr int EU = U::EU;
  constexpr int NT = ColwShape<WV>::kThreads;
  constexpr int UN = ColwShape<WV>::kUnroll;
  constexpr int WPB = WV;
  __shared__ __align__(16) Acc win[Win<Acc>::kElems];
  __shared__ Acc wl[kWinMaxM];
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int G = 1 << a.glog;
  const int P = kWave >> a.glog;
  const int q = lane >> a.glog;
  const int c = lane & (G - 1);
  const int M = (int)a.M;
  for (int i = threadIdx.x; i < M; i += NT) wl[i] = a.w[i];
  __syncthreads();
  const bool tl = a.tail > 0 && c == a.upr;
  const bool cu = c < a.upr || tl;
  const i64 eo = tl ? a.R - EU : (i64)c * EU;
  const int from = tl ? EU - a.tail : 0;
  const i64 rs = a.R * (i64)sizeof(T);
  const TaskRange tr = block_range((a.L + P - 1) / P);
  i64 org = 0, wbase = 0, wend = 0;
  for (i64 t0 = tr.begin; t0 < tr.end; t0 += WPB) {
    const i64 tlast = min(t0 + WPB, tr.end) - 1;
    const i64 ys = t0 * P * a.R;
    const i64 ye = min(a.L, (tlast + 1) * P) * a.R;
    if (t0 == tr.begin) {
      wbase = ys;
      org = win_origin(a.y, ys);
    } else if (ye - org > Win<Acc>::kElems) {
      win_flush<Acc, NT>(a.y, win, org, wbase, ys);
      wbase = ys;
      org = win_origin(a.y, ys);
    }
    wend = ye;
    const i64 g = t0 + wv;
    const i64 l = g * P + q;
    if (g > tlast || !cu || l >= a.L) continue;
    const char* base = (const char*)a.A + (l * a.M * a.R + eo) * (i64)sizeof(T);
    Acc acc[EU];
#pragma unroll
    for (int e = 0; e < EU; ++e) acc[e] = (Acc)0;
    int m = 0;
    // float64: the next UN rows' loads are issued before this batch is
    // summed, as in the column strips
    if constexpr (sizeof(Acc) == 8) {
      if (M >= UN) {
        typename U::Raw cur[UN];
#pragma unroll
        for (int k = 0; k < UN; ++k) cur[k] = U::load(base + (i64)k * rs, 0);
        for (; m + 2 * UN <= M; m += UN) {
          typename U::Raw nxt[UN];
#pragma unroll
          for (int k = 0; k < UN; ++k) nxt[k] = U::load(base + (i64)(m + UN + k) * rs, 0);
#pragma unroll
          for (int k = 0; k < UN; ++k) {
            Acc v[EU];
            U::unpack(cur[k], v);
            const Acc wk = wl[m + k];
#pragma unroll
            for (int e = 0; e < EU; ++e) acc[e] = fma(v[e], wk, acc[e]);
          }
#pragma unroll
          for (int k = 0; k < UN; ++k) cur[k] = nxt[k];
        }
#pragma unroll
        for (int k = 0; k < UN; ++k) {
          Acc v[EU];
          U::unpack(cur[k], v);
          const Acc wk = wl[m + k];
#pragma unroll
          for (int e = 0; e < EU; ++e) acc[e] = fma(v[e], wk, acc[e]);
        }
        m += UN;
      }
    }
    for (; m + UN <= M; m += UN) {
      typename U::Raw raw[UN];
#pragma unroll
      for (int k = 0; k < UN; ++k) raw[k] = U::load(base + (i64)(m + k) * rs, 0);
#pragma unroll
      for (int k = 0; k < UN; ++k) {
        Acc v[EU];
        U::unpack(raw[k], v);
        const Acc wk = wl[m + k];
#pragma unroll
        for (int e = 0; e < EU; ++e) acc[e] = fma(v[e], wk, acc[e]);
      }
    }
    if (m < M) {
      // the last M mod UN rows, loads issued together (M is uniform)
      typename U::Raw raw[UN - 1];
#pragma unroll
      for (int k = 0; k < UN - 1; ++k) raw[k] = m + k < M ? U::load(base + (i64)(m + k) * rs, 0) : U::zero();
#pragma unroll
      for (int k = 0; k < UN - 1; ++k) {
        if (m + k < M) {
          Acc v[EU];
          U::unpack(raw[k], v);
          const Acc wk = wl[m + k];
#pragma unroll
          for (int e = 0; e < EU; ++e) acc[e] = fma(v[e], wk, acc[e]);
        }
      }
    }
    const i64 idx = l * a.R + eo;
    Acc* wp = win + (idx - org);
#pragma unroll
    for (int e = 0; e < EU; ++e)
      if (e >= from) wp[e] = epilogue(acc[e], a.y, idx + e, l, a.alpha, a.beta, a.oscale, a.odiv);
  }
  if (tr.begin < tr.end) win_flush<Acc, NT>(a.y, win, org, wbase, wend);
}

// Short rows: the lane layout of k_row_short with UN rows per lane per task.
template <int DT, bool VEC, int ROLE>
__global__ __launch_bounds__(kRowswThreads) void k_rowsw(RowArgs<typename St<DT>::Acc> a) {
  typedef typename St<DT>::Acc Acc;
  typedef Unit<DT, VEC> U;
  constexpr int EU = U::EU;
  constexpr int UN = kRowswUnroll;
  constexpr int WPB = kRowswThreads / kWave;
  __shared__ __align__(16) Acc win[Win<Acc>::kElems];
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int G = 1 << a.glog;
  const int P = kWave >> a.glog;
  const int sub = lane & (G - 1);
  const int rsub = lane >> a.glog;
  const bool tl = a.tail > 0 && sub == a.upr;
  const bool active = sub < a.upr || tl;
  const i64 eo = tl ? a.ld - EU : (i64)sub * EU;
  const int from = tl ? EU - a.tail : 0;
  // Weights in registers; the elements of a ragged end that the last full
  // unit already covered, and every element of a lane past the row's
  // units, are weighted 0, so loads need no masks: an inactive lane reads
  // the row's first unit, a row past the end re-reads the last row, and
  // neither is stored (A is finite).
  Acc wk[EU];
  if (active) {
    load_w<Acc, EU>(a.w, eo, wk);
#pragma unroll
    for (int e = 0; e < EU; ++e)
      if (e < from) wk[e] = (Acc)0;
  } else {
#pragma unroll
    for (int e = 0; e < EU; ++e) wk[e] = (Acc)0;
  }
  const i64 eol = active ? eo : 0;
  const i64 per = (i64)P * UN;
  const TaskRange tr = block_range((a.L + per - 1) / per);
  auto load_task = [&](i64 t, typename U::Raw (&r)[UN]) {
#pragma unroll
    for (int k = 0; k < UN; ++k) {
      const i64 row = t * per + (i64)k * P + rsub;
      r[k] = U::load(a.A, (row < a.L ? row : a.L - 1) * a.ld + eol);
    }
  };
  // E4M3 spends 24 vector instructions on each 16-byte load: a wave loads
  // its next round's rows before summing this round's (same sums)
  constexpr bool PIPE = EU >= 16 || sizeof(Acc) == 8;
  typename U::Raw nxt[PIPE ? UN : 1];
  if constexpr (PIPE) {
    if (tr.begin + wv < tr.end) load_task(tr.begin + wv, nxt);
  }
  i64 org = 0, wbase = 0, wend = 0;
  for (i64 t0 = tr.begin; t0 < tr.end; t0 += WPB) {
    const i64 tlast = min(t0 + WPB, tr.end) - 1;
    const i64 ys = t0 * per;
    const i64 ye = min(a.L, (tlast + 1) * per);
    if (t0 == tr.begin) {
      wbase = ys;
      org = win_origin(a.y, ys);
    } else if (ye - org > Win<Acc>::kElems) {
      win_flush<Acc, kRowswThreads>(a.y, win, org, wbase, ys);
      wbase = ys;
      org = win_origin(a.y, ys);
    }
    wend = ye;
    const i64 t = t0 + wv;
    typename U::Raw raw[UN];
    if constexpr (PIPE) {
      // this round's rows were loaded in the last round; load the next's
#pragma unroll
      for (int k = 0; k < UN; ++k) raw[k] = nxt[k];
      if (t + WPB < tr.end) load_task(t + WPB, nxt);
      if (t > tlast) continue;
    } else {
      if (t > tlast) continue;
      load_task(t, raw);
    }
    const i64 base = t * per;
#pragma unroll
    for (int k = 0; k < UN; ++k) {
      Acc v[EU];
      U::unpack(raw[k], v);
      Acc s_ = (Acc)0;
#pragma unroll
      for (int e = 0; e < EU; ++e) s_ = fma(v[e], wk[e], s_);
      s_ = group_sum(s_, a.glog);
      const i64 row = base + (i64)k * P + rsub;
      if (sub == 0 && row < a.L)
        win[row - org] = epilogue(s_, a.y, row, row, a.alpha, a.beta, a.oscale, a.odiv);
    }
  }
  if (tr.begin < tr.end) win_flush<Acc, kRowswThreads>(a.y, win, org, wbase, wend);
}

// ---------------------------------------------------------------- kStage
// A slab l is the contiguous block A[l][0..M)[0..R) of E = M*R elements.  A
// workgroup takes blocks of sb consecutive slabs (sb*E elements, a multiple
// of 16 bytes, so every block starts 16-byte aligned): it copies a block
// into LDS with 16-byte loads, each of the NT threads holding kStageVecs/NT
// of them, issues the loads of its next block, and computes the current block's
// sb*R outputs from LDS while those loads are in flight.  G = 2^glog lanes
// per output group split the contracted extent and combine with shuffles.
// For 4- and 8-byte elements, when a slab row is a whole number of 16-byte
// words, an output group is the VE = 16 / element-size consecutive columns
// one LDS word holds, so each LDS read feeds VE accumulators.  Narrow
// formats read one dword (2 fp16 / bf16 or 4 E4M3 columns) when a slab row
// is a whole number of dwords, else one element: 16-byte words lost more
// to the wider groups' reductions and LDS bank conflicts than they gained
// (E4M3 32^6 mode 4: 37 -> 26% of peak), dwords gain (39 -> 53%).
// The M weights sit at the end of the staging buffer (the planner keeps the
// blocks clear of them): read from global memory inside the compute loop,
// each weight would wait behind the next block's loads, which are issued
// before the compute and complete in order.
constexpr int kStageBytes = 32768;
__host__ __device__ constexpr i64 stage_wres(i64 M, i64 acc_bytes) { return (M * acc_bytes + 15) / 16 * 16; }
// With the output window: staging buffer, window, threads per workgroup and
// workgroups per CU, by element size.  Measured on gfx950 over Table 1's
// staged modes: for 4- and 8-byte elements one 1024-thread workgroup per CU
// with a 64 KB staging buffer and a 64 KB window beats four 256-thread
// workgroups with 32 KB blocks and 8 KB windows by 5-10 points (float32
// 10^9 mode 7: 59 -> 66%, 13^8 mode 6: 61 -> 70%, float64 10^9 mode 7:
// 62 -> 69%), and a 96 KB window behind a 32 KB block loses 2-14; for E4M3
// (32^6 mode 4) the four small workgroups keep 8 points more.
struct StageCfg { int threads, bytes, win, bpc; };
__host__ __device__ constexpr StageCfg stage_cfg(int eb) {
  return eb >= 4 ? StageCfg{1024, 65536, 65536, 1} : StageCfg{256, 32768, 8192, 4};
}

template <typename Acc>
struct StageArgs {
  const void* A; const Acc* w; Acc* y;
  i64 L, M, R, sb, nblocks;
  int glog;
  Acc alpha, beta;
  const float* oscale; i64 odiv;
};

template <int DT, int ROLE, int VB, int NT, bool WIN>
__global__ __launch_bounds__(NT) void k_stage(StageArgs<typename St<DT>::Acc> a) {
  typedef typename St<DT>::Acc Acc;
  typedef typename St<DT>::T T;
  constexpr int EB = (int)sizeof(T);
  constexpr int VE = VB == 0 ? 1 : VB / EB;   // columns per output group
  constexpr StageCfg C = stage_cfg(EB);
  constexpr int kStageVecs = (WIN ? C.bytes : kStageBytes) / 16;
  constexpr int PER = kStageVecs / NT;        // 16-byte loads per thread per block
  constexpr int WE = C.win / (int)sizeof(Acc);
  __shared__ uint4 lds[kStageVecs];
  __shared__ __align__(16) Acc win[WIN ? WE : 1];
  const int tid = threadIdx.x;
  Acc* wl = (Acc*)((char*)lds + kStageVecs * 16 - stage_wres(a.M, sizeof(Acc)));
  for (i64 i = tid; i < a.M; i += NT) wl[i] = a.w[i];  // visible after the first block's barrier
  const i64 E = a.M * a.R;
  const int G = 1 << a.glog;
  const int sub = tid & (G - 1);
  // Within a block every index fits 32 bits (a block is at most the staging
  // buffer).  Output group o of a block is (slab ls, group rv) = o / Rv,
  // o % Rv; a thread steps o by S, so (ls, rv) advance by (S / Rv, S % Rv)
  // with one carry instead of a division per output.
  const int Rv = (int)(a.R / VE);  // output groups per slab row
  const int Ei = (int)E, Ri = (int)a.R, Mi = (int)a.M, dE = G * Ri;
  const int tot = (int)a.sb * Rv;
  const int S = NT >> a.glog;
  const int Sq = S / Rv, Sr = S % Rv;
  const int o0 = tid >> a.glog, ls0 = o0 / Rv, rv0 = o0 % Rv;
  uint4 r[PER];
  i64 nvec = 0;
  auto issue = [&](i64 b) {
    const i64 l0 = b * a.sb;
    const i64 ns = min(a.sb, a.L - l0);
    nvec = ns * E * EB / 16;
    const char* src = (const char*)a.A + l0 * E * EB;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const i64 v = tid + (i64)k * NT;
      r[k] = v < nvec ? stream_load16(src + v * 16) : uint4{0u, 0u, 0u, 0u};
    }
  };
  // with the window a workgroup takes a contiguous range of blocks (their
  // outputs are one stretch of y), else blocks are dealt round-robin
  const TaskRange tr = WIN ? block_range(a.nblocks) : block_tasks(a.nblocks);
  i64 org = 0, wbase = 0, wend = 0;
  i64 b = tr.begin;
  if (b < tr.end) issue(b);
  for (; b < tr.end; b += tr.step) {
    const i64 l0 = b * a.sb;
    const i64 ns = min(a.sb, a.L - l0);
    __syncthreads();  // the previous block's outputs no longer read the LDS
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const i64 v = tid + (i64)k * NT;
      if (v < nvec) lds[v] = r[k];
    }
    {  // bytes of the last block after its final whole 16-byte vector
      const i64 e0 = nvec * 16 / EB, e1 = ns * E;
      const T* src = (const T*)a.A + l0 * E;
      if (e0 + tid < e1) ((T*)lds)[e0 + tid] = src[e0 + tid];
    }
    __syncthreads();
    if (b + tr.step < tr.end) issue(b + tr.step);
    if constexpr (WIN) {
      const i64 ys = l0 * a.R, ye = (l0 + ns) * a.R;
      if (b == tr.begin) {
        wbase = ys;
        org = win_origin(a.y, ys);
      } else if (ye - org > WE) {
        win_flush<Acc, NT>(a.y, win, org, wbase, ys);
        wbase = ys;
        org = win_origin(a.y, ys);
      }
      wend = ye;
    }
    const int nout = (int)ns * Rv;
    const T* sl = (const T*)lds;
    int ls = ls0, rv = rv0;
    for (int o = o0; o < tot; o += S) {
      Acc acc[4][VE];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < VE; ++v) acc[j][v] = (Acc)0;
      if (o < nout) {
        auto step = [&](int e, int m, Acc* ac) {
          Acc val[VE];
          if constexpr (VB == 16) {
            unpack16<DT>(*(const uint4*)(sl + e), val);
          } else if constexpr (VB == 4) {
            unpack4<DT>(*(const uint32_t*)(sl + e), val);
          } else {
            val[0] = load_elem<DT>(sl, e);
          }
          const Acc wm = wl[m];
#pragma unroll
          for (int v = 0; v < VE; ++v) ac[v] = fma(val[v], wm, ac[v]);
        };
        int m = sub;
        int e = ls * Ei + rv * VE + sub * Ri;
        for (; m + 3 * G < Mi; m += 4 * G, e += 4 * dE) {
          step(e, m, acc[0]);
          step(e + dE, m + G, acc[1]);
          step(e + 2 * dE, m + 2 * G, acc[2]);
          step(e + 3 * dE, m + 3 * G, acc[3]);
        }
        for (; m < Mi; m += G, e += dE) step(e, m, acc[0]);
      }
#pragma unroll
      for (int v = 0; v < VE; ++v) {
        Acc t = (acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v]);
        for (int off = G >> 1; off >= 1; off >>= 1) t += shfl_xor(t, off);
        if (sub == 0 && o < nout) {
          const i64 idx = l0 * a.R + (i64)o * VE + v;
          const Acc out = epilogue(t, a.y, idx, l0 + ls, a.alpha, a.beta, a.oscale, a.odiv);
          if constexpr (WIN) win[idx - org] = out;
          else a.y[idx] = out;
        }
      }
      ls += Sq;
      rv += Sr;
      if (rv >= Rv) {
        rv -= Rv;
        ++ls;
      }
    }
  }
  if constexpr (WIN) {
    if (tr.begin < tr.end) win_flush<Acc, NT>(a.y, win, org, wbase, wend);
  }
}

// ---------------------------------------------------------------- finalize
// y[i] = epilogue(sum_{s < nsplit} part[s * n + i]) in split order.
template <typename Acc, int ROLE>
__global__ __launch_bounds__(kBlock) void k_finalize(const Acc* part, Acc* y, i64 n, int nsplit,
                                                     i64 R, Acc alpha, Acc beta,
                                                     const float* oscale, i64 odiv) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (i64)gridDim.x * blockDim.x) {
    Acc s = (Acc)0;
    for (int k = 0; k < nsplit; ++k) s += part[(i64)k * n + i];
    y[i] = epilogue(s, y, i, i / R, alpha, beta, oscale, odiv);
  }
}

// Few outputs, many splits: a workgroup owns 64 outputs and its 8 waves sum
// interleaved subsets of the splits; the 8 partials are combined in wave
// order (a fixed order, so the result does not depend on scheduling).
constexpr int kFinWaves = 8;

template <typename Acc, int ROLE>
__global__ __launch_bounds__(kFinWaves * kWave) void k_finalize_wide(const Acc* part, Acc* y, i64 n,
                                                                   int nsplit, i64 R, Acc alpha,
                                                                   Acc beta, const float* oscale,
                                                                   i64 odiv) {
  __shared__ Acc red[kFinWaves][kWave];
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  for (i64 tile = blockIdx.x; tile * kWave < n; tile += gridDim.x) {
    const i64 i = tile * kWave + lane;
    Acc a0 = (Acc)0, a1 = (Acc)0, a2 = (Acc)0, a3 = (Acc)0;
    if (i < n) {
      int k = w;
      for (; k + 3 * kFinWaves < nsplit; k += 4 * kFinWaves) {
        a0 += part[(i64)k * n + i];
        a1 += part[(i64)(k + kFinWaves) * n + i];
        a2 += part[(i64)(k + 2 * kFinWaves) * n + i];
        a3 += part[(i64)(k + 3 * kFinWaves) * n + i];
      }
      for (; k < nsplit; k += kFinWaves) a0 += part[(i64)k * n + i];
    }
    red[w][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (w == 0 && i < n) {
      Acc s = (Acc)0;
#pragma unroll
      for (int q = 0; q < kFinWaves; ++q) s += red[q][lane];
      y[i] = epilogue(s, y, i, i / R, alpha, beta, oscale, odiv);
    }
    __syncthreads();
  }
}

// Reduce nsplit partial rows of n outputs into y with the epilogue.
template <typename Acc, int ROLE>
hipError_t launch_finalize(const Acc* part, Acc* y, i64 n, int nsplit, i64 R, Acc alpha, Acc beta,
                           const float* oscale, i64 odiv, hipStream_t st) {
  const i64 cap = 4 * (i64)device_cus();
  if (nsplit >= 32 && n <= 64 * cap) {
    const int g = (int)std::max<i64>(1, std::min<i64>((n + kWave - 1) / kWave, cap));
    hipLaunchKernelGGL((k_finalize_wide<Acc, ROLE>), dim3(g), dim3(kFinWaves * kWave), 0, st, part, y,
                       n, nsplit, R, alpha, beta, oscale, odiv);
  } else {
    const int g = (int)std::max<i64>(1, std::min<i64>((n + kBlock - 1) / kBlock, cap));
    hipLaunchKernelGGL((k_finalize<Acc, ROLE>), dim3(g), dim3(kBlock), 0, st, part, y, n, nsplit, R,
                       alpha, beta, oscale, odiv);
  }
  return hipGetLastError();
}

// ====================================================================== host
namespace {

int ceil_log2(i64 v) {
  int g = 0;
  while (((i64)1 << g) < v) ++g;
  return g;
}

i64 cdiv(i64 a, i64 b) { return (a + b - 1) / b; }

#ifndef TVC_WIN_BPC
#define TVC_WIN_BPC 1
#endif
constexpr bool kWinOn = kWinBytes > 0;
constexpr int kWinBlocksPerCu = TVC_WIN_BPC;    // workgroups per CU with a window

// The output window pays where y is a sizeable share of the traffic (short
// contracted extents) and every workgroup gets several rounds of wave tasks.
bool win_ok(i64 M, i64 wave_tasks) {
  return kWinOn && !tuning().win_off && M <= kWinMaxM && wave_tasks >= 16 * (i64)device_cus();
}

int grid_for(i64 blocks_needed, int family, int default_bpc) {
  int bpc = tuning().blocks_per_cu[family] > 0 ? tuning().blocks_per_cu[family] : default_bpc;
  i64 cap = (i64)bpc * device_cus();
  return (int)std::max<i64>(1, std::min<i64>(blocks_needed, cap));
}

}  // namespace

namespace {

i64 gcd_(i64 a, i64 b) {
  while (b) {
    const i64 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

TvcPlan plan_tvc(int dtype, i64 L, i64 M, i64 R, bool a4, bool w4, bool a16) {
  TvcPlan p;
  const i64 b = (i64)elem_bytes(dtype);
  const i64 epv = 16 / b;
  const size_t ab = acc_bytes(dtype);
  const int waves_per_block = kBlock / kWave;
  // 16-byte units need every row of the contiguous extent to hold at least
  // one unit, and rows of 4- and 8-byte elements to start on a dword
  // boundary; rows of 1- and 2-byte formats may start on any byte (odd
  // lengths), since global loads need no alignment (bf16 30623^2, E4M3
  // 13^8 and the like: one element per lane otherwise, 10-30% of peak).  A
  // ragged end (len mod EPV elements) is one more unit.
  const i64 len = R == 1 ? M : R;
  p.vec = a4 && (R != 1 || w4) && ((len * b) % 4 == 0 || b < 4) && len >= epv;
  p.upr = p.vec ? len / epv : len;
  p.tail = p.vec ? (int)(len % epv) : 0;
  const i64 nu = p.upr + (p.tail > 0 ? 1 : 0);
  // Small slabs: stage whole slabs through LDS where the slab kernel loses
  // coalescing (measured on gfx950 over the Table 1 shapes): slabs of at
  // most 4 KB whose right extent is ragged, not a power of two, or at most
  // 2 units wide (4 in float64: 8^10 mode 8, 64-byte slab rows, 64 -> 71%;
  // float32 rows of that width, 16^7 mode 5, lose 77 -> 68% staged), or
  // narrower than one 16-byte vector (where a slab lane would load one
  // element: E4M3 8^10 mode 8, 8-byte rows, 16% of peak).  Other
  // power-of-two slab widths stay with the slab kernel, which is faster
  // there.  Rows (R == 1) of 33-64 units are staged only in
  // float64, where the row kernel's double accumulators limit occupancy;
  // in the other formats the row kernel is 10-40% faster on them.  Rows
  // narrower than one 16-byte vector are staged in every format (the row
  // kernel would load them one element per lane: E4M3 8^10 mode 9, 8-byte
  // rows, 8% of peak).  A block of sb slabs must be a multiple of 16 bytes.
  const i64 sbytes = M * R * b;
  const bool pow2 = (nu & (nu - 1)) == 0;
  const bool small = R == 1 ? ((dtype == TVC_F64 && p.vec && nu > 32 && nu <= 64) || (!p.vec && sbytes < 16))
                            : (sbytes <= 4096 && nu <= 32 && (p.tail > 0 || !pow2 || nu <= 2 || (b == 8 && nu <= 4) || !p.vec));
  if (a16 && small && !tuning().stage_off) {
    const i64 q = 16 / gcd_(16, sbytes);
    // Slabs per block in a staging buffer of the given size less the
    // weights.  Where the weights displace slabs from a block whose outputs
    // were a whole number of 256-byte stretches, keep them so (measured on
    // 8^10 mode 8, 256-byte slabs: 127 slabs per block, 54%; 120, 66%): the
    // window's flushes otherwise end inside cache lines.
    const i64 wres = stage_wres(M, ab);
    const i64 ob = R * (i64)ab;  // output bytes per slab
    auto slabs = [&](i64 bytes) {
      const i64 full = (bytes / sbytes) / q * q;
      const i64 s = ((bytes - wres) / sbytes) / q * q;
      if (s == full || full * ob % 256 != 0) return s;
      const i64 g = 256 / gcd_(256, ob);
      const i64 q2 = q / gcd_(q, g) * g;
      const i64 s2 = ((bytes - wres) / sbytes) / q2 * q2;
      return s2 >= 1 ? s2 : s;
    };
    // with many blocks, outputs through the LDS window (a block's outputs at
    // most half of it), in blocks of the window variant's staging size
    const StageCfg sc = stage_cfg((int)b);
    const i64 sbw = slabs(sc.bytes);
    const bool win = kWinOn && !tuning().win_off && sbw >= 1 &&
                     cdiv(L, sbw) >= 4 * (i64)device_cus() && sbw * R * (i64)ab <= sc.win / 2;
    const i64 sb = win ? sbw : slabs(kStageBytes);
    if (sb >= 1) {
      p.family = kStage;
      p.win = win;
      p.sb = sb;
      p.vec = true;
      // LDS word per read: 16 bytes for 4- and 8-byte elements when a slab
      // row is a whole number of them, a dword for narrower ones when a row
      // is a whole number of dwords, else one element
      p.stage_vb = (b >= 4 && (R * b) % 16 == 0) ? 16 : (b < 4 && (R * b) % 4 == 0) ? 4 : 0;
      const i64 ve = p.stage_vb == 0 ? 1 : p.stage_vb / b;
      p.nsplit = 1;
      p.tasks = cdiv(L, sb);
      p.grid = grid_for(p.tasks, kStage, p.win ? sc.bpc : 4);
      const int nt = p.win ? sc.threads : kBlock;
      // lanes per output group: as many as keep all threads busy
      // (measured: a whole wave per row serialises the reductions)
      const i64 outs = std::max<i64>(sb * R / ve, 1);
      int g = 0;
      while (g < 6 && ((i64)2 << g) * outs <= nt && ((i64)1 << g) < M) ++g;
      p.glog = g;
      p.part_bytes = 0;
      return p;
    }
  }
  if (R == 1) {
    p.family = kRow;
    if (nu > 32) {
      p.lng = true;
      // RB rows share each weight load and a lane keeps 8/RB units of each
      // in flight, 8 loads in all.  A row that fits one pass of the wave
      // (q = ceil(upr / 64) <= 8/RB units per lane) keeps its weights in
      // registers: take the largest such RB.  Longer rows take RB = 2 (4
      // contiguous units per row per step stream better than 8 rows of one
      // unit), except when the weight vector is far larger than the L2
      // (over 8 MB, the HOPM pass 1 of high orders): then every group of RB
      // rows re-reads it from beyond the L2, and RB = 8 cuts that traffic 4x.
      // Measured on gfx950 over the Table 1 and 32^6 sweeps.
      const i64 q = cdiv(p.upr, kWave);
      int rb = 1;
      if (q <= 4) {
        rb = q <= 1 ? 8 : (q <= 2 ? 4 : 2);
      } else if (dtype == TVC_F64 && q <= 8) {
        // float64 rows of 5-8 units per lane: one row per wave with its
        // weights in registers and the next row's loads in flight
        rb = 1;
      } else {
        rb = (M * (i64)acc_bytes(dtype) > ((i64)8 << 20)) ? 8 : 2;
      }
      while (rb > 1 && L < rb) rb /= 2;
      p.rb = rb;
      const i64 groups = cdiv(L, p.rb);
      p.nsplit = 1;
      p.chunk = p.upr;
      // lanes address a chunk with 32-bit byte offsets: at most 2^31 bytes
      const i64 max_chunk = ((i64)1 << 31) / (p.vec ? 16 : b);
      // Few long rows: split each row so that enough waves stream at once.
      const i64 want = 8 * (i64)device_cus();
      const i64 ku = 8 / p.rb;
      if (groups < want && p.upr >= 2 * kWave * ku) {
        i64 ns = std::min<i64>(cdiv(2 * want, groups), p.upr / (kWave * ku));
        ns = std::max<i64>(ns, 1);
        i64 chunk = cdiv(p.upr, ns);
        chunk = cdiv(chunk, kWave) * kWave;
        p.chunk = chunk;
        p.nsplit = (int)cdiv(p.upr, chunk);
      }
      if (p.chunk > max_chunk) {
        p.chunk = max_chunk;  // a multiple of the wave width
        p.nsplit = (int)cdiv(p.upr, p.chunk);
      }
      p.tasks = groups * p.nsplit;
      p.grid = grid_for(cdiv(p.tasks, waves_per_block), kRow, 16);
    } else {
      p.lng = false;
      p.glog = ceil_log2(std::max<i64>(nu, 1));
      const i64 per = (i64)(kWave >> p.glog) * kShortUnroll;
      p.tasks = cdiv(L, per);
      p.grid = grid_for(cdiv(p.tasks, waves_per_block), kRow, 4);
      const i64 wtasks = cdiv(L, (i64)(kWave >> p.glog) * kRowswUnroll);
      if (win_ok(M, wtasks)) {
        p.win = true;
        p.tasks = wtasks;
        p.grid = grid_for(cdiv(p.tasks, kRowswThreads / kWave), kRow, kWinBlocksPerCu);
      }
    }
  } else {
    if (nu > 32) {
      p.family = kCol;
      int sm = tuning().split_m > 0 ? tuning().split_m : (M >= 8 ? 4 : 1);
      if (sm != 1 && sm != 2 && sm != 4) sm = 4;
      p.splitm = sm;
      const i64 tc = kBlock / sm;
      const i64 ctiles = cdiv(nu, tc);
      const i64 tasks = L * ctiles;
      p.nsplit = 1;
      p.chunk = M;
      const i64 want = 4 * (i64)device_cus();
      // Splits of M: about two rounds of the grid's workgroups.  Up to
      // 4-byte elements at most two, so that no round runs nearly empty
      // (30623^2 mode 0, 120 column tiles: 2160 -> 2040 tasks for 1024
      // workgroups, 72 -> 74.6% of peak); float64 keeps the next split up
      // (240 tiles: 2160 tasks 75.5%, 1920 tasks 72.7%)
      if (tasks < want && M >= (i64)sm * kUnroll * 8) {
        const i64 ns0 = b == 8 ? cdiv(2 * want, tasks) : 2 * want / tasks;
        i64 ns = std::min<i64>(ns0, M / ((i64)sm * kUnroll * 4));
        ns = std::max<i64>(ns, 1);
        p.chunk = cdiv(M, ns);
        p.nsplit = (int)cdiv(M, p.chunk);
      }
      p.tasks = tasks * p.nsplit;
      p.grid = grid_for(p.tasks, kCol, 4);
      // Column strips (no split of M, weights fit in LDS): the widest strip
      // up to 4 units per lane that the rows fill and that still gives a
      // busy wave per SIMD (with the window: several rounds per workgroup);
      // short M also writes through the LDS window (one workgroup per CU
      // beside it), a round of strips being at most half the window.
      if (p.nsplit == 1 && M <= kColwMaxM && !tuning().strips_off) {
        const bool win = win_ok(M, L * cdiv(nu, kWave));
        // 8 waves of 4 loads for short strips (M < 32); with the window (one
        // workgroup per CU) E4M3, whose 16 conversions and FMAs per load need
        // more waves and loads in flight to hide them, takes 16 waves of 4
        // loads and one unit per lane (32^6 modes 1-3: 54-58% with 4 waves,
        // 65-67% with 8, 70-74% with 16; 8^10 mode 5 41 -> 51%)
        const int wv = (win && epv >= 16 && p.vec) ? 16 : (M < 32 || (win && epv >= 16)) ? 8 : 4;
        // with the window, 4 units per lane where rows are a multiple of
        // 64 KB apart and less than 64 MB (measured on 32^6: float32 mode 1,
        // 4 MB rows, 75 -> 79%, bf16 mode 2, 64 KB rows, 81 -> 86%; 4 KB rows
        // and 64-128 MB rows lose 2-4% with 4); else, for M >= 32, 2 (Table
        // 1's odd row pitches, one unit per lane against two: float64 63^5
        // modes 0-1 71 -> 80%, 175^4 mode 1 78 -> 83%, float32 63^5 mode 1
        // 79 -> 83%; 32^6 modes 0 and 3 even; 4 loses 1-3 points on
        // float32 and bf16) or 4 for float64 rows that are not a multiple
        // of 4 KB apart (63^5 modes 0-2 80 -> 82-85%, 175^4 mode 1 83 ->
        // 84%, mode 0 83 -> 82%); 1 for shorter M, where 2 lost (10^9
        // modes 0-4 75 -> 71%, 8^10 mode 1 77 -> 71%)
        const i64 pitch = R * b;
        const int cmax = !win ? 4
                         : (pitch % 65536 == 0 && pitch < ((i64)64 << 20)) ? 4
                         : M < 32 ? 1
                         : (b == 8 && pitch % 4096 != 0) ? 4 : 2;
        for (int cpt = cmax; cpt >= 1; cpt /= 2) {
          const i64 strips = L * cdiv(nu, (i64)kWave * cpt);
          const bool fits = !win || (i64)wv * kWave * cpt * epv * (i64)ab <= kWinBytes / 2;
          const i64 need = (win ? 16 : wv) * (i64)device_cus();
          if ((cpt == 1 || nu >= (i64)kWave * cpt) && strips >= need && fits) {
            p.strips = true;
            p.win = win;
            p.wv = wv;
            p.cpt = cpt;
            // rotated row order for rows 1-64 MB apart with 4 units per lane
            p.mrot = win && cpt == 4 && pitch >= ((i64)1 << 20);
            p.tasks = strips;
            p.grid = grid_for(cdiv(strips, wv), kCol, win ? kWinBlocksPerCu : 4);
            break;
          }
        }
      }
    } else {
      p.family = kSlab;
      p.glog = ceil_log2(std::max<i64>(nu, 1));
      const i64 P = kWave >> p.glog;
      const i64 groups = cdiv(L, P);
      p.nsplit = 1;
      p.chunk = M;
      const i64 want = 16 * (i64)device_cus();
      if (groups < want && M >= (i64)kSlabUnroll * 16) {
        i64 ns = std::min<i64>(cdiv(2 * want, groups), M / ((i64)kSlabUnroll * 8));
        ns = std::max<i64>(ns, 1);
        p.chunk = cdiv(M, ns);
        p.nsplit = (int)cdiv(M, p.chunk);
      }
      p.tasks = groups * p.nsplit;
      p.grid = grid_for(cdiv(p.tasks, waves_per_block), kSlab, 4);
      if (p.nsplit == 1 && win_ok(M, groups)) {
        p.win = true;
        // 8 waves for short slabs and for the 2- and 1-byte formats, whose
        // slab rows are narrower (32^6 bf16 mode 4: 76 -> 77.5%)
        p.wv = (M < 32 || b < 4) ? 8 : 4;
        p.grid = grid_for(cdiv(p.tasks, p.wv), kSlab, kWinBlocksPerCu);
      }
    }
  }
  p.part_bytes = p.nsplit > 1 ? align256((size_t)p.nsplit * (size_t)(L * R) * ab) : 0;
  return p;
}

namespace {

// The column-strip kernel for a plan: vector or scalar units, waves per
// workgroup, column units per lane, window.
template <int DT, int ROLE, bool VEC, int WV, int CPT>
void launch_colw_c(const TvcPlan& p, dim3 grd, hipStream_t st, const ColArgs<typename St<DT>::Acc>& a) {
  const dim3 blk(ColwShape<WV>::kThreads);
  if (p.win) hipLaunchKernelGGL((k_colw<DT, VEC, ROLE, WV, CPT, true>), grd, blk, 0, st, a);
  else hipLaunchKernelGGL((k_colw<DT, VEC, ROLE, WV, CPT, false>), grd, blk, 0, st, a);
}

template <int DT, int ROLE, bool VEC, int WV>
void launch_colw_w(const TvcPlan& p, dim3 grd, hipStream_t st, const ColArgs<typename St<DT>::Acc>& a) {
  if (p.cpt == 4) launch_colw_c<DT, ROLE, VEC, WV, 4>(p, grd, st, a);
  else if (p.cpt == 2) launch_colw_c<DT, ROLE, VEC, WV, 2>(p, grd, st, a);
  else launch_colw_c<DT, ROLE, VEC, WV, 1>(p, grd, st, a);
}

template <int DT, int ROLE>
void launch_colw(const TvcPlan& p, dim3 grd, hipStream_t st, const ColArgs<typename St<DT>::Acc>& a) {
  if constexpr (DT == TVC_F8E4M3) {
    if (p.vec && p.wv == 16) {
      launch_colw_c<DT, ROLE, true, 16, 1>(p, grd, st, a);
      return;
    }
  }
  if (p.vec) {
    if (p.wv == 8) launch_colw_w<DT, ROLE, true, 8>(p, grd, st, a);
    else launch_colw_w<DT, ROLE, true, 4>(p, grd, st, a);
  } else {
    if (p.wv == 8) launch_colw_w<DT, ROLE, false, 8>(p, grd, st, a);
    else launch_colw_w<DT, ROLE, false, 4>(p, grd, st, a);
  }
}

template <int DT, int ROLE>
hipError_t run_dt(const void* A, i64 L, i64 M, i64 R, const void* w_, void* y_, double alpha,
                  double beta, const float* oscale, i64 odiv, const TvcPlan& p, void* part_,
                  hipStream_t st) {
  typedef typename St<DT>::Acc Acc;
  const Acc* w = (const Acc*)w_;
  Acc* y = (Acc*)y_;
  Acc* part = (Acc*)part_;
  const dim3 blk(kBlock);
  const dim3 grd(p.grid);
  if (p.family == kStage) {
    StageArgs<Acc> a{A, w, y, L, M, R, p.sb, p.tasks, p.glog, (Acc)alpha, (Acc)beta, oscale, odiv};
    constexpr int VW = (DT == TVC_F32 || DT == TVC_F64) ? 16 : 4;
    if (p.win) {
      constexpr int NT = stage_cfg((int)sizeof(typename St<DT>::T)).threads;
      const dim3 wblk(NT);
      if (p.stage_vb != 0 && p.stage_vb == VW)
        hipLaunchKernelGGL((k_stage<DT, ROLE, VW, NT, true>), grd, wblk, 0, st, a);
      else hipLaunchKernelGGL((k_stage<DT, ROLE, 0, NT, true>), grd, wblk, 0, st, a);
    } else {
      if (p.stage_vb != 0 && p.stage_vb == VW)
        hipLaunchKernelGGL((k_stage<DT, ROLE, VW, kBlock, false>), grd, blk, 0, st, a);
      else hipLaunchKernelGGL((k_stage<DT, ROLE, 0, kBlock, false>), grd, blk, 0, st, a);
    }
    return hipGetLastError();
  }
  if (p.family == kRow) {
    RowArgs<Acc> a{A, w, y, part, L, p.upr, p.chunk, p.nsplit, p.glog, (Acc)alpha, (Acc)beta,
                   oscale, odiv, 1, 0, M, p.tail};
    if (p.lng) {
      if (p.vec) {
        if (p.rb == 8) hipLaunchKernelGGL((k_row_long<DT, true, 8, ROLE>), grd, blk, 0, st, a);
        else if (p.rb == 4) hipLaunchKernelGGL((k_row_long<DT, true, 4, ROLE>), grd, blk, 0, st, a);
        else if (p.rb == 2) hipLaunchKernelGGL((k_row_long<DT, true, 2, ROLE>), grd, blk, 0, st, a);
        else hipLaunchKernelGGL((k_row_long<DT, true, 1, ROLE>), grd, blk, 0, st, a);
      } else {
        if (p.rb == 8) hipLaunchKernelGGL((k_row_long<DT, false, 8, ROLE>), grd, blk, 0, st, a);
        else if (p.rb == 4) hipLaunchKernelGGL((k_row_long<DT, false, 4, ROLE>), grd, blk, 0, st, a);
        else if (p.rb == 2) hipLaunchKernelGGL((k_row_long<DT, false, 2, ROLE>), grd, blk, 0, st, a);
        else hipLaunchKernelGGL((k_row_long<DT, false, 1, ROLE>), grd, blk, 0, st, a);
      }
    } else if (p.win) {
      const dim3 wblk(kRowswThreads);
      if (p.vec) hipLaunchKernelGGL((k_rowsw<DT, true, ROLE>), grd, wblk, 0, st, a);
      else hipLaunchKernelGGL((k_rowsw<DT, false, ROLE>), grd, wblk, 0, st, a);
    } else {
      if (p.vec) hipLaunchKernelGGL((k_row_short<DT, true, ROLE>), grd, blk, 0, st, a);
      else hipLaunchKernelGGL((k_row_short<DT, false, ROLE>), grd, blk, 0, st, a);
    }
  } else {
    const i64 tc = (p.family == kCol && p.strips) ? (i64)kWave * p.cpt : kBlock / p.splitm;
    const i64 nu = p.upr + (p.tail > 0 ? 1 : 0);
    ColArgs<Acc> a{A, w, y, part, L, M, p.upr, R, (nu + tc - 1) / tc, p.chunk, p.nsplit,
                   p.glog, (Acc)alpha, (Acc)beta, oscale, odiv, p.tail, p.mrot ? 1 : 0};
    if (p.family == kCol) {
      if (p.strips) {
        launch_colw<DT, ROLE>(p, grd, st, a);
      } else if (p.vec) {
        if (p.splitm == 4) hipLaunchKernelGGL((k_col<DT, true, 4, ROLE>), grd, blk, 0, st, a);
        else if (p.splitm == 2) hipLaunchKernelGGL((k_col<DT, true, 2, ROLE>), grd, blk, 0, st, a);
        else hipLaunchKernelGGL((k_col<DT, true, 1, ROLE>), grd, blk, 0, st, a);
      } else {
        if (p.splitm == 4) hipLaunchKernelGGL((k_col<DT, false, 4, ROLE>), grd, blk, 0, st, a);
        else if (p.splitm == 2) hipLaunchKernelGGL((k_col<DT, false, 2, ROLE>), grd, blk, 0, st, a);
        else hipLaunchKernelGGL((k_col<DT, false, 1, ROLE>), grd, blk, 0, st, a);
      }
    } else if (p.win) {
      if (p.wv == 8) {
        const dim3 wblk(ColwShape<8>::kThreads);
        if (p.vec) hipLaunchKernelGGL((k_slabw<DT, true, ROLE, 8>), grd, wblk, 0, st, a);
        else hipLaunchKernelGGL((k_slabw<DT, false, ROLE, 8>), grd, wblk, 0, st, a);
      } else {
        const dim3 wblk(ColwShape<4>::kThreads);
        if (p.vec) hipLaunchKernelGGL((k_slabw<DT, true, ROLE, 4>), grd, wblk, 0, st, a);
        else hipLaunchKernelGGL((k_slabw<DT, false, ROLE, 4>), grd, wblk, 0, st, a);
      }
    } else {
      if (p.vec) hipLaunchKernelGGL((k_slab<DT, true, ROLE>), grd, blk, 0, st, a);
      else hipLaunchKernelGGL((k_slab<DT, false, ROLE>), grd, blk, 0, st, a);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.nsplit > 1)
    e = launch_finalize<Acc, ROLE>((const Acc*)part, y, L * R, p.nsplit, R, (Acc)alpha, (Acc)beta,
                                   oscale, odiv, st);
  return e;
}

}  // namespace

namespace {

// Rows of length M whose weights change with the row: row i uses
// w + (i / wdiv) * wstride.  Only the row family; one row per wave task.
template <int DT>
hipError_t run_rows_pw_dt(const void* A, i64 L, i64 M, const void* w_, i64 wdiv, i64 wstride,
                          void* y_, const float* oscale, i64 odiv, const TvcPlan& p, void* part_,
                          hipStream_t st) {
  typedef typename St<DT>::Acc Acc;
  RowArgs<Acc> a{A, (const Acc*)w_, (Acc*)y_, (Acc*)part_, L, p.upr, p.chunk, p.nsplit, p.glog,
                 (Acc)1, (Acc)0, oscale, odiv, wdiv, wstride, M, p.tail};
  const dim3 blk(kBlock), grd(p.grid);
  constexpr int RW = kRoleRowWeights;
  if (p.lng) {
    if (p.vec) {
      if (p.rb == 8) hipLaunchKernelGGL((k_row_long<DT, true, 8, RW>), grd, blk, 0, st, a);
      else if (p.rb == 4) hipLaunchKernelGGL((k_row_long<DT, true, 4, RW>), grd, blk, 0, st, a);
      else if (p.rb == 2) hipLaunchKernelGGL((k_row_long<DT, true, 2, RW>), grd, blk, 0, st, a);
      else hipLaunchKernelGGL((k_row_long<DT, true, 1, RW>), grd, blk, 0, st, a);
    } else {
      if (p.rb == 8) hipLaunchKernelGGL((k_row_long<DT, false, 8, RW>), grd, blk, 0, st, a);
      else if (p.rb == 4) hipLaunchKernelGGL((k_row_long<DT, false, 4, RW>), grd, blk, 0, st, a);
      else if (p.rb == 2) hipLaunchKernelGGL((k_row_long<DT, false, 2, RW>), grd, blk, 0, st, a);
      else hipLaunchKernelGGL((k_row_long<DT, false, 1, RW>), grd, blk, 0, st, a);
    }
  } else {
    if (p.vec) hipLaunchKernelGGL((k_row_short<DT, true, RW>), grd, blk, 0, st, a);
    else hipLaunchKernelGGL((k_row_short<DT, false, RW>), grd, blk, 0, st, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.nsplit == 1) return e;
  return launch_finalize<Acc, RW>((const Acc*)part_, (Acc*)y_, L, p.nsplit, (i64)1, (Acc)1, (Acc)0,
                                  oscale, odiv, st);
}

}  // namespace

TvcPlan plan_rows_pw(int dtype, i64 L, i64 M, bool a4, bool w4, i64 wdiv) {
  TvcPlan p = plan_tvc(dtype, L, M, 1, a4, w4, false);
  if (p.win) {
    // row-dependent weights: the plain short-row kernel
    p.win = false;
    p.tasks = cdiv(L, (i64)(kWave >> p.glog) * kShortUnroll);
    p.grid = grid_for(cdiv(p.tasks, kBlock / kWave), kRow, 4);
  }
  if (p.lng) {
    // RB rows of a wave share one weight row: RB must divide wdiv (row
    // groups start at multiples of RB)
    int rb = p.rb;
    while (rb > 1 && (wdiv % rb) != 0) rb /= 2;
    if (rb != p.rb) {
      p.rb = rb;
      p.tasks = cdiv(L, rb) * p.nsplit;
      p.grid = grid_for(cdiv(p.tasks, kBlock / kWave), kRow, 16);
    }
  }
  return p;
}

hipError_t run_rows_pw(int dtype, const void* A, i64 L, i64 M, const void* w, i64 wdiv,
                       i64 wstride, void* y, const float* oscale, i64 odiv, const TvcPlan& p,
                       void* part, hipStream_t st) {
  switch (dtype) {
    case TVC_F64: return run_rows_pw_dt<TVC_F64>(A, L, M, w, wdiv, wstride, y, oscale, odiv, p, part, st);
    case TVC_F32: return run_rows_pw_dt<TVC_F32>(A, L, M, w, wdiv, wstride, y, oscale, odiv, p, part, st);
    case TVC_F16: return run_rows_pw_dt<TVC_F16>(A, L, M, w, wdiv, wstride, y, oscale, odiv, p, part, st);
    case TVC_BF16: return run_rows_pw_dt<TVC_BF16>(A, L, M, w, wdiv, wstride, y, oscale, odiv, p, part, st);
    case TVC_F8E4M3: return run_rows_pw_dt<TVC_F8E4M3>(A, L, M, w, wdiv, wstride, y, oscale, odiv, p, part, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t run_tvc(int dtype, const void* A, i64 L, i64 M, i64 R, const void* w, void* y,
                   double alpha, double beta, const float* oscale, i64 odiv, const TvcPlan& p,
                   void* part, hipStream_t st, int role) {
#define TVC_RUN(D)                                                                               \
  return role == kRoleHopm                                                                       \
             ? run_dt<D, kRoleHopm>(A, L, M, R, w, y, alpha, beta, oscale, odiv, p, part, st)   \
             : run_dt<D, kRoleContract>(A, L, M, R, w, y, alpha, beta, oscale, odiv, p, part, st)
  switch (dtype) {
    case TVC_F64: TVC_RUN(TVC_F64);
    case TVC_F32: TVC_RUN(TVC_F32);
    case TVC_F16: TVC_RUN(TVC_F16);
    case TVC_BF16: TVC_RUN(TVC_BF16);
    case TVC_F8E4M3: TVC_RUN(TVC_F8E4M3);
    default: return hipErrorInvalidValue;
  }
#undef TVC_RUN
}

tvc_status tvc_run_auto(int dtype, const void* A, i64 L, i64 M, i64 R, const void* w, void* y,
                        double alpha, double beta, const float* oscale, i64 odiv, void* ws,
                        size_t ws_bytes, hipStream_t st, int role) {
  const bool a4 = ((uintptr_t)A % 4) == 0;
  const bool w4 = ((uintptr_t)w % 4) == 0;
  const bool a16 = ((uintptr_t)A % 16) == 0;
  TvcPlan p = plan_tvc(dtype, L, M, R, a4, w4, a16);
  if (p.part_bytes > ws_bytes || (p.part_bytes > 0 && ws == nullptr))
    return fail(TVC_EWORKSPACE, "internal contraction needs " + std::to_string(p.part_bytes) +
                                    " workspace bytes");
  hipError_t e = run_tvc(dtype, A, L, M, R, w, y, alpha, beta, oscale, odiv, p, ws, st, role);
  if (e != hipSuccess) return fail(TVC_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
  return TVC_OK;
}

}  // namespace tvc
