// Batched HOPM: many independent float32 instances of uneven order and
// shape, all swept `sweeps` times by one persistent kernel.
//
// Each sweep of an instance follows the two-pass schedule of hopm.hip
// (Sec. 3 HOPM in the update order of Algorithm 1) and is split into four
// phases:
//   P1 (tiled)   rows [t*TR1, (t+1)*TR1) of M = A[n0 n1][R1] . (x_2 (x) ... (x) x_{d-1})
//   S1 (single)  x_0 <- M x_1 / ||.||, x_1 <- M^T x_0 / ||.||, w2 = x_0 (x) x_1
//   P2 (tiled)   partial_t[r] = sum over rows of tile t of w2[row] A[row, r]
//   S2 (single)  W_2 = sum_t partial_t; Algorithm 1's W chain for j >= 2 with
//                normalisation; the Kronecker weights of the next sweep.
// Work items (instance, phase, tile, sweep) live in a device queue.  A
// workgroup claims the next slot, waits until that slot has been
// published, and runs the item; the workgroup that completes the last tile
// of a phase (a per-instance counter) publishes the next phase.  No
// workgroup ever waits on a barrier with another, so progress does not
// depend on how many workgroups are resident; every wait is bounded and
// reports an error instead of hanging.  Partial sums are combined in tile
// order, so the results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "common.h"
#include "internal.h"

#define TVC_BATCH_MAX_ORDER 8

namespace tvc {

struct BatchDesc {           // mirrors hopm_batch_desc in include/tvc.h
  const float* A;
  double* x;
  int64_t dims[TVC_BATCH_MAX_ORDER];
  int32_t order;
  int32_t tile_rows1;
  int32_t tile_rows2;
  int32_t nt1;
  int32_t nt2;
  int32_t reserved;
  int64_t ws_offset;
  int64_t init_slot;
};

struct Item {
  int32_t inst, phase, tile, sweep;
};

enum { kP1 = 0, kS1 = 1, kP2 = 2, kS2 = 3 };

// Global header at the start of the workspace.
struct BatchHeader {
  uint32_t head;
  uint32_t tail;
  uint32_t done;
  uint32_t error;
  // profile of the last run (wall clock ticks summed over workgroups):
  // items run, ticks waiting for slots, ticks running items of each phase
  unsigned long long items, wait_ticks, work_ticks[4];
};

constexpr int kBThreads = 256;
constexpr int kSpinLimit = 1 << 24;   // ~ seconds of short sleeps before giving up

// Per-instance scratch (floats), 16-byte aligned pieces.
struct InstLayout {
  int64_t wv, w1, M, w2, part, Wa, Wb, Ca, Cb, y, total;   // offsets in floats
  int64_t woff[TVC_BATCH_MAX_ORDER];
  int64_t off[TVC_BATCH_MAX_ORDER];
  int64_t n01, R1, nsum, nmax;
};

__host__ __device__ inline int64_t round4(int64_t v) { return (v + 3) & ~(int64_t)3; }

__host__ __device__ inline void inst_layout_to(InstLayout& L, const int64_t* n, int d, int nt2) {
  int64_t o = 0, ws = 0, xs = 0;
  L.nmax = 0;
  for (int m = 0; m < d; ++m) {
    L.woff[m] = ws;
    L.off[m] = xs;
    ws += round4(n[m]);
    xs += n[m];
    L.nmax = n[m] > L.nmax ? n[m] : L.nmax;
  }
  L.nsum = xs;
  L.n01 = n[0] * n[1];
  L.R1 = 1;
  int64_t nmin = INT64_MAX;
  for (int m = 2; m < d; ++m) {
    L.R1 *= n[m];
    nmin = n[m] < nmin ? n[m] : nmin;
  }
  L.wv = o; o += round4(ws);
  L.w1 = o; o += round4(L.R1);
  L.M = o; o += round4(L.n01);
  L.w2 = o; o += round4(L.n01);
  L.part = o; o += round4((int64_t)nt2 * L.R1);
  L.Wa = o; o += round4(L.R1);
  L.Wb = o; o += round4(L.R1);
  const int64_t c = d >= 4 ? L.R1 / nmin : 1;
  L.Ca = o; o += round4(c);
  L.Cb = o; o += round4(c);
  L.y = o; o += round4(L.nmax);
  L.total = o;
}

__host__ __device__ inline InstLayout inst_layout(const int64_t* n, int d, int nt2) {
  InstLayout L{};
  inst_layout_to(L, n, d, nt2);
  return L;
}

// ---------------------------------------------------------------- helpers
__device__ inline float block_sum_f(float v, float* sh) {
  v = wave_sum(v);
  if (lane_id() == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  float s = 0.f;
  for (int w = 0; w < kBThreads / kWave; ++w) s += sh[w];
  __syncthreads();
  return s;
}

__device__ inline double block_sum_d(double v, double* sh) {
  v = wave_sum(v);
  if (lane_id() == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kBThreads / kWave; ++w) s += sh[w];
  __syncthreads();
  return s;
}

// x_j <- y / ||y|| (double), mirror into wv; returns ||y|| and the change.
__device__ void wg_normalize(const float* y, int64_t n, double* x, float* wv, double* sh,
                             double* nrm_out, double* delta_out, int* degenerate) {
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBThreads) ss += (double)y[i] * (double)y[i];
  ss = block_sum_d(ss, sh);
  const double nrm = sqrt(ss);
  *nrm_out = nrm;
  if (!(nrm > 0.0) || !isfinite(nrm)) {
    *degenerate = 1;
    *delta_out = 0.0;
    return;
  }
  const double inv = 1.0 / nrm;
  double dd = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBThreads) {
    const double v = (double)y[i] * inv;
    const double df = v - x[i];
    dd += df * df;
    x[i] = v;
    wv[i] = (float)v;
  }
  dd = block_sum_d(dd, sh);
  *delta_out = sqrt(dd);
}

// dst[l*R + r] = sum_m src[(l*M + m)*R + r] * w[m]  (small tensors, one workgroup)
__device__ void wg_contract(const float* src, int64_t L, int64_t M, int64_t R, const float* w,
                            float* dst) {
  const int64_t n = L * R;
  for (int64_t o = threadIdx.x; o < n; o += kBThreads) {
    const int64_t l = o / R, r = o - l * R;
    const float* p = src + l * M * R + r;
    float acc = 0.f;
    for (int64_t m = 0; m < M; ++m) acc = fmaf(p[m * R], w[m], acc);
    dst[o] = acc;
  }
}

// Kronecker product of the double vectors of modes [m0, m1) into w (float).
__device__ void wg_kron(const double* x, const InstLayout& L, const int64_t* n, int m0, int m1,
                        float* w) {
  int64_t total = 1;
  for (int m = m0; m < m1; ++m) total *= n[m];
  if (total <= (int64_t)UINT32_MAX) {
    for (int64_t r = threadIdx.x; r < total; r += kBThreads) {
      uint32_t rem = (uint32_t)r;
      double p = 1.0;
      for (int m = m1 - 1; m >= m0; --m) {
        const uint32_t nm = (uint32_t)n[m];
        const uint32_t q = rem / nm;
        p *= x[L.off[m] + (rem - q * nm)];
        rem = q;
      }
      w[r] = (float)p;
    }
    return;
  }
  for (int64_t r = threadIdx.x; r < total; r += kBThreads) {
    int64_t rem = r;
    double p = 1.0;
    for (int m = m1 - 1; m >= m0; --m) {
      const int64_t i = rem % n[m];
      rem /= n[m];
      p *= x[L.off[m] + i];
    }
    w[r] = (float)p;
  }
}

// Queue flags and counters are polled with relaxed agent-scope loads (they
// read the coherent copy without touching the caches); the one acquire fence
// after a successful poll makes the producer's data visible.  On a chip whose
// L2 is split across dies, an agent-scope acquire invalidates the local L2,
// so it must not sit inside a polling loop.
__device__ inline uint32_t relaxed_load_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish `count` items (instance inst, phase, tiles 0..count-1, sweep).
// Called by the whole workgroup.
__device__ void wg_push(BatchHeader* hdr, Item* items, uint32_t* flags, int64_t slots, int inst,
                        int phase, int count, int sweep, uint32_t* sh_slot) {
  __syncthreads();
  if (threadIdx.x == 0) *sh_slot = atomicAdd(&hdr->tail, (uint32_t)count);
  __syncthreads();
  const uint32_t s0 = *sh_slot;
  if ((int64_t)s0 + count > slots) {            // accounting error: never write past the queue
    if (threadIdx.x == 0) atomicOr(&hdr->error, 2u);
    __syncthreads();
    return;
  }
  for (int t = threadIdx.x; t < count; t += kBThreads) items[s0 + t] = Item{inst, phase, t, sweep};
  // one release for the whole workgroup: everything it wrote (phase results
  // and the items) is visible before any flag is
  __syncthreads();
  if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  for (int t = threadIdx.x; t < count; t += kBThreads)
    __hip_atomic_store(&flags[s0 + t], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
}

// Count a finished tile; true for the workgroup that finished the last one.
__device__ bool wg_tile_done(uint32_t* counter, int ntiles, uint32_t* sh_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // this tile's results
    const uint32_t old = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool last = old == (uint32_t)(ntiles - 1);
    if (last) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every other tile's
      __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    *sh_flag = last ? 1u : 0u;
  }
  __syncthreads();
  return *sh_flag != 0;
}

// A pointer every lane holds the same value of (read from LDS), moved to
// scalar registers.
// Tile bytes in the global address space: the tensor pointers come from a
// descriptor in memory, so without the address space the compiler issues
// flat loads, which also count against the LDS counter (every LDS wait of
// the window and the row-group combine then waits for them too).
typedef const __attribute__((address_space(1))) char gchar;
typedef const __attribute__((address_space(1))) u32x4u gu32x4;
__device__ __forceinline__ uint4 tile_load16(gchar* p) {
  const u32x4u v = __builtin_nontemporal_load((gu32x4*)p);
  uint4 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

__device__ __forceinline__ const char* uniform_ptr(const void* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const char*)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------- phases
// Rows [r0, r1) of a float matrix with R columns: 16-byte loads at dword
// alignment (row starts are 4-byte aligned), the ragged end of a row read as
// one more unit over its last 4 columns with the overlap dropped.

// Outputs of a tile are collected in an LDS window of kBWin floats and
// written in bursts: small stores spread through a read stream cost HBM
// several times their bytes (pass-1 rows of 16-256 values make M up to
// 1/16 of the tile's bytes, pass-2 partials of order-5 instances up to 1/25).
constexpr int kBWin = 8192;

__device__ __forceinline__ void bwin_flush(float* dst, const float* win, int n) {
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBThreads) dst[i] = win[i];
  __syncthreads();
}

// P1: M[row] = sum_c A[row, c] * w1[c].  G lanes per row (a power of two,
// at most 64), several row groups in flight per wave; the rows of a tile go
// in chunks of kBWin through the window.
__device__ void phase_p1(const BatchDesc& D, const InstLayout& L, float* s, int tile, float* win) {
  const int64_t R = L.R1;
  const int64_t r0 = (int64_t)tile * D.tile_rows1;
  const int64_t r1 = min(L.n01, r0 + D.tile_rows1);
  const float* w = s + L.w1;
  float* M = s + L.M;
  if (R < 4) {
    for (int64_t row = r0 + threadIdx.x; row < r1; row += kBThreads) {
      float acc = 0.f;
      for (int64_t c = 0; c < R; ++c) acc = fmaf(D.A[row * R + c], w[c], acc);
      M[row] = acc;
    }
    return;
  }
  constexpr int RU = 8;  // row groups in flight per wave
  constexpr int NW = kBThreads / kWave;
  const int64_t U = R / 4;
  const int T = (int)(R % 4);
  const int64_t nu = U + (T ? 1 : 0);
  int g = 0;
  while (((int64_t)1 << g) < nu && g < 6) ++g;
  const int G = 1 << g, P = kWave >> g;
  const int lane = lane_id();
  const int sub = lane & (G - 1), rsub = lane >> g;
  const int wave = threadIdx.x / kWave;
  // the tile is far below 2^31 bytes: lanes address it with 32-bit offsets
  gchar* tbase = (gchar*)uniform_ptr(D.A + r0 * R);
  for (int64_t c0 = r0; c0 < r1; c0 += kBWin) {
    const int64_t c1 = min(r1, c0 + kBWin);
    for (int64_t rb = c0 + (int64_t)wave * P * RU; rb < c1; rb += (int64_t)NW * P * RU) {
      float acc[RU];
#pragma unroll
      for (int j = 0; j < RU; ++j) acc[j] = 0.f;
      for (int64_t u = sub; u < nu; u += G) {
        const bool tl = T != 0 && u == U;
        const int64_t e = tl ? R - 4 : u * 4;
        const int from = tl ? 4 - T : 0;
        float wt[4];
        load_w<float, 4>(w, e, wt);
        uint4 raw[RU];
#pragma unroll
        for (int j = 0; j < RU; ++j) {
          // rows past the window's end re-read its last row (never stored):
          // no branch per load
          int64_t row = rb + (int64_t)j * P + rsub;
          row = row < c1 ? row : c1 - 1;
          raw[j] = tile_load16(tbase + (uint32_t)(((row - r0) * R + e) * 4));
        }
#pragma unroll
        for (int j = 0; j < RU; ++j) {
          float v[4];
          unpack16<TVC_F32>(raw[j], v);
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (q >= from) acc[j] = fmaf(v[q], wt[q], acc[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const float v = group_sum(acc[j], g);
        const int64_t row = rb + (int64_t)j * P + rsub;
        if (sub == 0 && row < c1) win[row - c0] = v;
      }
    }
    bwin_flush(M + c0, win, (int)(c1 - c0));
  }
}

// P2: part[c] = sum over the tile's rows of w2[row] * A[row, c].  TC threads
// per row own 16-byte column units, the 256/TC row groups of the workgroup
// stream interleaved rows and combine in LDS in a fixed order; the partials
// go in chunks of kBWin columns through the window.
__device__ void phase_p2(const BatchDesc& D, const InstLayout& L, float* s, int tile, float* lds,
                         float* win) {
  const int64_t R = L.R1;
  const int64_t r0 = (int64_t)tile * D.tile_rows2;
  const int64_t r1 = min(L.n01, r0 + D.tile_rows2);
  const float* w2 = s + L.w2;
  float* part = s + L.part + (int64_t)tile * R;
  if (R < 4) {
    for (int64_t c = threadIdx.x; c < R; c += kBThreads) {
      float acc = 0.f;
      for (int64_t row = r0; row < r1; ++row) acc = fmaf(w2[row], D.A[row * R + c], acc);
      part[c] = acc;
    }
    return;
  }
  constexpr int UN = 8;  // rows in flight per thread
  const int64_t U = R / 4;
  const int T = (int)(R % 4);
  const int64_t nu = U + (T ? 1 : 0);
  int g = 0;
  while (((int64_t)1 << g) < nu && g < 8) ++g;
  const int TC = 1 << g, RG = kBThreads >> g;
  const int tc = threadIdx.x & (TC - 1), rg = threadIdx.x >> g;
  gchar* tbase = (gchar*)uniform_ptr(D.A + r0 * R);   // 32-bit lane offsets below
  int64_t wc0 = 0;  // first column held by the window
  for (int64_t cb = 0; cb < nu; cb += TC) {
    if ((cb + TC) * 4 - wc0 > kBWin) {  // this block's columns would not fit
      bwin_flush(part + wc0, win, (int)(cb * 4 - wc0));
      wc0 = cb * 4;
    }
    const int64_t u = cb + tc;
    const bool on = u < nu;
    const bool tl = T != 0 && u == U;
    // lanes past the row's units load its last unit (never stored)
    const int64_t e = tl || !on ? R - 4 : u * 4;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int64_t row = r0 + rg; row < r1; row += (int64_t)RG * UN) {
      uint4 raw[UN];
      float wr[UN];
#pragma unroll
      for (int k = 0; k < UN; ++k) {
        const int64_t rk = row + (int64_t)k * RG;
        const bool ok = rk < r1;
        // rows past the tile re-read its last row with weight 0 (A is finite)
        const int64_t rc = ok ? rk : r1 - 1;
        raw[k] = tile_load16(tbase + (uint32_t)(((rc - r0) * R + e) * 4));
        const float wk = w2[rc];
        wr[k] = ok ? wk : 0.f;
      }
#pragma unroll
      for (int k = 0; k < UN; ++k) {
        float v[4];
        unpack16<TVC_F32>(raw[k], v);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = fmaf(v[q], wr[k], acc[q]);
      }
    }
    if (RG > 1) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) lds[(rg * TC + tc) * 4 + q] = acc[q];
      __syncthreads();
      if (rg == 0)
        for (int h = 1; h < RG; ++h)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] += lds[(h * TC + tc) * 4 + q];
    }
    if (rg == 0 && on) {
      const int from = tl ? 4 - T : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q >= from) win[e + q - wc0] = acc[q];
    }
  }
  bwin_flush(part + wc0, win, (int)(R - wc0));
}

__device__ void phase_s1(const BatchDesc& D, const InstLayout& L, float* s, double* sh,
                         float* lds, hopm_stats* st) {
  const int64_t* n = D.dims;
  const int64_t n0 = n[0], n1 = n[1];
  const float* M = s + L.M;
  float* wv = s + L.wv;
  float* y = s + L.y;
  double nrm, dl;
  int degen = 0;
  // y0 = M x1: a wave per row of M
  const int wave = threadIdx.x / kWave, lane = lane_id();
  for (int64_t i = wave; i < n0; i += kBThreads / kWave) {
    float a = 0.f;
    for (int64_t k = lane; k < n1; k += kWave) a = fmaf(M[i * n1 + k], wv[L.woff[1] + k], a);
    a = wave_sum(a);
    if (lane == 0) y[i] = a;
  }
  __syncthreads();
  wg_normalize(y, n0, D.x + L.off[0], wv + L.woff[0], sh, &nrm, &dl, &degen);
  double delta = dl;
  __syncthreads();
  // y1 = M^T x0: threads over columns, 4 row groups combined in LDS
  for (int64_t cb = 0; cb < n1; cb += kWave) {
    const int64_t c = cb + lane;
    float a = 0.f;
    if (c < n1)
      for (int64_t i = wave; i < n0; i += kBThreads / kWave) a = fmaf(M[i * n1 + c], wv[L.woff[0] + i], a);
    lds[threadIdx.x] = a;
    __syncthreads();
    if (wave == 0 && c < n1) y[c] = lds[lane] + lds[kWave + lane] + lds[2 * kWave + lane] + lds[3 * kWave + lane];
    __syncthreads();
  }
  wg_normalize(y, n1, D.x + L.off[1], wv + L.woff[1], sh, &nrm, &dl, &degen);
  delta = fmax(delta, dl);
  __syncthreads();
  // w2 = x0 (x) x1 for pass 2
  wg_kron(D.x, L, n, 0, 2, s + L.w2);
  if (threadIdx.x == 0) {
    st->delta = delta;
    if (degen) st->status = TVC_EDEGENERATE;
  }
}

__device__ void phase_s2(const BatchDesc& D, const InstLayout& L, float* s, double* sh,
                         hopm_stats* st) {
  const int64_t* n = D.dims;
  const int d = D.order;
  float* wv = s + L.wv;
  float* Wa = s + L.Wa;
  // W_2 = sum of the pass-2 partials in tile order
  for (int64_t r = threadIdx.x; r < L.R1; r += kBThreads) {
    float acc = 0.f;
    for (int t = 0; t < D.nt2; ++t) acc += s[L.part + (int64_t)t * L.R1 + r];
    Wa[r] = acc;
  }
  __syncthreads();
  float* Wcur = Wa;
  float* Woth = s + L.Wb;
  int64_t wsize = L.R1;
  double delta = 0.0, nrm = 0.0, dl;
  int degen = 0;
  for (int j = 2; j < d; ++j) {
    if (j > 2) {
      wg_contract(Wcur, 1, n[j - 1], wsize / n[j - 1], wv + L.woff[j - 1], Woth);
      __syncthreads();
      wsize /= n[j - 1];
      float* t = Wcur;
      Wcur = Woth;
      Woth = t;
    }
    const float* src = Wcur;
    int64_t t = wsize;
    int bi = 0;
    for (int m = d - 1; m > j; --m) {
      float* dst = (m == j + 1) ? s + L.y : (bi ? s + L.Cb : s + L.Ca);
      wg_contract(src, t / n[m], n[m], 1, wv + L.woff[m], dst);
      __syncthreads();
      t /= n[m];
      src = dst;
      bi ^= 1;
    }
    wg_normalize(src, n[j], D.x + L.off[j], wv + L.woff[j], sh, &nrm, &dl, &degen);
    delta = fmax(delta, dl);
    __syncthreads();
  }
  // Kronecker weights of the next pass 1
  wg_kron(D.x, L, n, 2, d, s + L.w1);
  if (threadIdx.x == 0) {
    st->delta = fmax(st->delta, delta);
    st->lambda = nrm;
    st->sweeps += 1;
    if (degen) st->status = TVC_EDEGENERATE;
  }
}

// ---------------------------------------------------------------- kernels
__global__ void k_batch_clear(BatchHeader* hdr, uint32_t* counters, int count, uint32_t* flags,
                              int64_t slots) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < slots;
       i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    counters[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hdr->head = 0u;
    hdr->tail = 0u;
    hdr->done = 0u;
    hdr->error = 0u;
    hdr->items = 0ull;
    hdr->wait_ticks = 0ull;
    for (int q = 0; q < 4; ++q) hdr->work_ticks[q] = 0ull;
  }
}

// One workgroup per instance: mirror the vectors, first Kronecker weights,
// stats reset, and the pass-1 items of sweep 0 at the instance's slots.
__global__ __launch_bounds__(kBThreads) void k_batch_init(const BatchDesc* descs, int count,
                                                          char* ws, Item* items, uint32_t* flags,
                                                          hopm_stats* stats, BatchHeader* hdr,
                                                          int64_t initial) {
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const BatchDesc D = descs[i];
    const InstLayout L = inst_layout(D.dims, D.order, D.nt2);
    float* s = (float*)(ws + D.ws_offset);
    for (int m = 0; m < D.order; ++m)
      for (int64_t k = threadIdx.x; k < D.dims[m]; k += kBThreads)
        s[L.wv + L.woff[m] + k] = (float)D.x[L.off[m] + k];
    wg_kron(D.x, L, D.dims, 2, D.order, s + L.w1);
    if (threadIdx.x == 0) {
      stats[i].lambda = 0.0;
      stats[i].delta = 0.0;
      stats[i].sweeps = 0;
      stats[i].status = TVC_OK;
      stats[i].refine_sweeps = 0;
      stats[i].reserved = 0;
    }
    for (int t = threadIdx.x; t < D.nt1; t += kBThreads) {
      items[D.init_slot + t] = Item{i, kP1, t, 0};
      flags[D.init_slot + t] = 1u;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) hdr->tail = (uint32_t)initial;
}

__global__ __launch_bounds__(kBThreads) void k_batch_run(const BatchDesc* descs, int count, int sweeps,
                                                         char* ws, Item* items, uint32_t* flags,
                                                         uint32_t* counters, hopm_stats* stats,
                                                         BatchHeader* hdr, int64_t slots) {
  __shared__ double sh[kBThreads / kWave];
  __shared__ float lds[4 * kBThreads];
  __shared__ float win[kBWin];
  __shared__ uint32_t sh_u[2];
  __shared__ Item sh_item;
  __shared__ BatchDesc sh_desc;
  __shared__ InstLayout sh_layout;
  // thread 0's running totals: items run, ticks spent claiming and waiting
  // for a slot, ticks spent running items (added to the header at exit)
  unsigned long long n_items = 0ull, t_wait = 0ull, t_mark = 0ull;
  unsigned long long t_work[4] = {0ull, 0ull, 0ull, 0ull};
  for (;;) {
    if (threadIdx.x == 0) {
      t_mark = wall_clock64();
      const uint32_t h = atomicAdd(&hdr->head, 1u);
      uint32_t ok = 0u;
      if ((int64_t)h < slots) {
        int spins = 0;
        uint32_t f;
        while ((f = relaxed_load_u32(&flags[h])) == 0u) {
          if (relaxed_load_u32(&hdr->error) != 0u || ++spins > kSpinLimit) break;
          __builtin_amdgcn_s_sleep(4);
        }
        if (f != 0u) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          ok = 1u;
          sh_item = items[h];
        } else {
          atomicOr(&hdr->error, 1u);
        }
      }
      sh_u[0] = ok;
      const unsigned long long now = wall_clock64();
      t_wait += now - t_mark;
      t_mark = now;
    }
    __syncthreads();
    if (sh_u[0] == 0u) {
      if (threadIdx.x == 0) {
        atomicAdd(&hdr->items, n_items);
        atomicAdd(&hdr->wait_ticks, t_wait);
        for (int q = 0; q < 4; ++q) atomicAdd(&hdr->work_ticks[q], t_work[q]);
      }
      return;
    }
    const Item it = sh_item;
    // the instance's descriptor and scratch layout, once per item, in LDS
    // (their arrays are indexed by mode at run time)
    if (threadIdx.x == 0) {
      sh_desc = descs[it.inst];
      inst_layout_to(sh_layout, sh_desc.dims, sh_desc.order, sh_desc.nt2);
    }
    __syncthreads();
    const BatchDesc& D = sh_desc;
    const InstLayout& L = sh_layout;
    float* s = (float*)(ws + D.ws_offset);
    hopm_stats* st = stats + it.inst;
    if (it.phase == kP1) {
      phase_p1(D, L, s, it.tile, win);
      if (wg_tile_done(&counters[it.inst], D.nt1, &sh_u[1]))
        wg_push(hdr, items, flags, slots, it.inst, kS1, 1, it.sweep, &sh_u[1]);
    } else if (it.phase == kS1) {
      phase_s1(D, L, s, sh, lds, st);
      wg_push(hdr, items, flags, slots, it.inst, kP2, D.nt2, it.sweep, &sh_u[1]);
    } else if (it.phase == kP2) {
      phase_p2(D, L, s, it.tile, lds, win);
      if (wg_tile_done(&counters[it.inst], D.nt2, &sh_u[1]))
        wg_push(hdr, items, flags, slots, it.inst, kS2, 1, it.sweep, &sh_u[1]);
    } else {
      phase_s2(D, L, s, sh, st);
      if (it.sweep + 1 < sweeps) {
        wg_push(hdr, items, flags, slots, it.inst, kP1, D.nt1, it.sweep + 1, &sh_u[1]);
      } else if (threadIdx.x == 0) {
        atomicAdd(&hdr->done, 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      ++n_items;
      const unsigned long long dt = wall_clock64() - t_mark;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q == it.phase) t_work[q] += dt;
    }
  }
}

static size_t header_bytes(int count, int64_t slots) {
  return align256(sizeof(BatchHeader)) + align256((size_t)count * 4) + align256((size_t)slots * sizeof(Item)) +
         align256((size_t)slots * 4);
}

}  // namespace tvc

using namespace tvc;

static_assert(sizeof(hopm_batch_desc) == sizeof(tvc::BatchDesc), "descriptor layouts differ");

extern "C" {

int32_t hopm_batch_prepare(hopm_batch_desc* descs, int32_t count, int32_t sweeps, int32_t tile_elems,
                           hopm_batch_plan* plan) {
  if (!descs || !plan || count < 1 || sweeps < 1) return fail(TVC_EINVAL, "bad batch arguments");
  if (tile_elems < 1) tile_elems = 1 << 16;
  int64_t slots = 0, initial = 0;
  for (int i = 0; i < count; ++i) {
    hopm_batch_desc& d = descs[i];
    if (d.order < 3 || d.order > TVC_BATCH_MAX_ORDER)
      return fail(TVC_EINVAL, "instance " + std::to_string(i) + ": order outside [3, 8]");
    if (!d.A || !d.x) return fail(TVC_EINVAL, "instance " + std::to_string(i) + ": NULL pointer");
    if ((uintptr_t)d.A % 4 || (uintptr_t)d.x % 8)
      return fail(TVC_EINVAL, "instance " + std::to_string(i) + ": misaligned pointer");
    int64_t n01 = 1, R1 = 1;
    for (int m = 0; m < d.order; ++m) {
      if (d.dims[m] < 1 || d.dims[m] > (1 << 20))
        return fail(TVC_EINVAL, "instance " + std::to_string(i) + ": bad dim");
      if (m < 2) n01 *= d.dims[m];
      else R1 *= d.dims[m];
    }
    if (n01 * R1 > ((int64_t)1 << 34)) return fail(TVC_EINVAL, "instance too large");
    if (d.tile_rows1 < 1) d.tile_rows1 = (int32_t)std::max<int64_t>(1, tile_elems / R1);
    if (d.tile_rows2 < 1) d.tile_rows2 = (int32_t)std::max<int64_t>(1, tile_elems / R1);
    d.nt1 = (int32_t)((n01 + d.tile_rows1 - 1) / d.tile_rows1);
    d.nt2 = (int32_t)((n01 + d.tile_rows2 - 1) / d.tile_rows2);
    d.init_slot = initial;
    initial += d.nt1;
    slots += (int64_t)sweeps * (d.nt1 + d.nt2 + 2);
  }
  if (slots > (int64_t)UINT32_MAX / 2) return fail(TVC_EINVAL, "too many work items");
  size_t off = header_bytes(count, slots);
  for (int i = 0; i < count; ++i) {
    hopm_batch_desc& d = descs[i];
    InstLayout L = inst_layout(d.dims, d.order, d.nt2);
    d.ws_offset = (int64_t)off;
    off += align256((size_t)L.total * 4);
  }
  plan->count = count;
  plan->sweeps = sweeps;
  plan->queue_slots = slots;
  plan->initial_items = initial;
  plan->ws_bytes = off;
  return TVC_OK;
}

int32_t hopm_batch_run(const hopm_batch_desc* d_descs, const hopm_batch_plan* plan, int32_t grid,
                       void* ws, size_t ws_bytes, hopm_stats* d_stats, void* stream) {
  if (!d_descs || !plan || !d_stats) return fail(TVC_EINVAL, "NULL argument");
  if (!ws || ws_bytes < plan->ws_bytes || (uintptr_t)ws % 256)
    return fail(TVC_EWORKSPACE, "batch workspace of " + std::to_string(plan->ws_bytes) + " bytes required");
  if (plan->count < 1 || plan->sweeps < 1 || plan->queue_slots < 1)
    return fail(TVC_EINVAL, "plan not prepared");
  if (grid <= 0) grid = 4 * device_cus();
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  BatchHeader* hdr = (BatchHeader*)w;
  size_t o = align256(sizeof(BatchHeader));
  uint32_t* counters = (uint32_t*)(w + o);
  o += align256((size_t)plan->count * 4);
  Item* items = (Item*)(w + o);
  o += align256((size_t)plan->queue_slots * sizeof(Item));
  uint32_t* flags = (uint32_t*)(w + o);
  const BatchDesc* D = (const BatchDesc*)d_descs;
  const int gc = (int)std::min<int64_t>((plan->queue_slots + 255) / 256, 8 * (int64_t)device_cus());
  hipLaunchKernelGGL(k_batch_clear, dim3(std::max(gc, 1)), dim3(256), 0, s, hdr, counters, plan->count,
                     flags, plan->queue_slots);
  hipLaunchKernelGGL(k_batch_init, dim3(std::min(plan->count, 4 * device_cus())), dim3(kBThreads), 0,
                     s, D, plan->count, w, items, flags, d_stats, hdr, plan->initial_items);
  hipLaunchKernelGGL(k_batch_run, dim3(grid), dim3(kBThreads), 0, s, D, plan->count, plan->sweeps, w,
                     items, flags, counters, d_stats, hdr, plan->queue_slots);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(TVC_EHIP, hipGetErrorString(e));
  return TVC_OK;
}

int32_t hopm_batch_profile(const void* ws, uint64_t* d_out, void* stream) {
  if (!ws || !d_out) return fail(TVC_EINVAL, "NULL argument");
  hipError_t e = hipMemcpyAsync(d_out, &((const BatchHeader*)ws)->items, 6 * sizeof(uint64_t),
                                hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return fail(TVC_EHIP, hipGetErrorString(e));
  return TVC_OK;
}

int32_t hopm_batch_error(const void* ws, uint32_t* d_error_out, void* stream) {
  if (!ws || !d_error_out) return fail(TVC_EINVAL, "NULL argument");
  hipError_t e = hipMemcpyAsync(d_error_out, &((const BatchHeader*)ws)->error, 4,
                                hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return fail(TVC_EHIP, hipGetErrorString(e));
  return TVC_OK;
}

}  // extern "C"
