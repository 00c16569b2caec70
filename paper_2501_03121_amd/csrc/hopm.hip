// Higher-order power method on one device (Sec. 3 canonical HOPM, update
// order of Algorithm 1).
//
// One sweep performs the external iterations j = 0..d-1 in order; iteration
// j replaces x_j by the normalised contraction of A with every other vector,
// using the vectors already refreshed in this sweep (Gauss-Seidel).
//
// Schedule (d >= 3).  Algorithm 1 streams the full tensor twice per sweep
// (A x_1 x_1 at j = 0 and A x_0 x_0 at j = 1) and reuses the buffer W for
// j >= 2.  Here the two full passes are arranged so that nothing of size
// N / n_k is written between them:
//   pass 1:  M = A contracted with x_2 (x) ... (x) x_{d-1}   (an n_0 x n_1
//            matrix; A is read as [n_0 n_1][n_2 ... n_{d-1}] rows)
//            j = 0:  x_0 <- normalise(M x_1)
//            j = 1:  x_1 <- normalise(M^T x_0)
//   pass 2:  W_2 = A contracted with x_0 (x) x_1            (A read as one
//            [n_0 n_1] x [n_2 ... n_{d-1}] slab)
//            j >= 2: W_j = W_{j-1} x_{j-1} x_{j-1} (Algorithm 1's reuse of W),
//                    x_j <- normalise(W_j contracted with x_{j+1}..x_{d-1})
// Both j = 0 and j = 1 of Algorithm 1 contract A with exactly these vectors
// (contraction order does not change the result), so the iterates are those
// of the paper's sweep; only the intermediates differ.  d = 2 is two plain
// matrix-vector products per sweep.
//
// Vectors are kept in double (the master copy) and mirrored in the
// accumulation type for the contraction kernels.  Norms, the Rayleigh
// quotient lambda = ||y_{d-1}|| and the change delta are computed in double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <functional>
#include <string>
#include <vector>

#include "common.h"
#include "internal.h"

namespace tvc {

constexpr int kNormBlock = 1024;

// ---------------------------------------------------------------- kernels
struct VecOffsets {
  int d;
  i64 n[TVC_MAX_ORDER];
  i64 off[TVC_MAX_ORDER];
  i64 woff[TVC_MAX_ORDER];
};

// Mirror the double vectors into the accumulation type (16-byte aligned per
// vector) and reset the stats record.
template <typename Acc>
__global__ void k_prepare(const double* x, Acc* wv, VecOffsets vo, hopm_stats* st) {
  for (int m = 0; m < vo.d; ++m)
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < vo.n[m];
         i += (i64)gridDim.x * blockDim.x)
      wv[vo.woff[m] + i] = (Acc)x[vo.off[m] + i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->lambda = 0.0;
    st->delta = 0.0;
    st->sweeps = 0;
    st->status = TVC_OK;
    st->refine_sweeps = 0;
    st->reserved = 0;
  }
}

__device__ __forceinline__ double block_sum_1024(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < kNormBlock / kWave) s = sh[threadIdx.x];
  if (threadIdx.x < kWave) s = wave_sum(s);
  __syncthreads();
  if (threadIdx.x == 0) sh[0] = s;
  __syncthreads();
  s = sh[0];
  __syncthreads();
  return s;
}

// kNoMirror (small-step programs of Jacobi sweeps): update x but not its
// accumulation-type mirror, which the sweep's remaining contractions still
// read as the previous vectors; a final mirror step copies x over.
enum { kFirstJ = 1, kLastJ = 2, kAlignSign = 4, kNoMirror = 8 };

// x <- y / ||y||, mirrored into wv; delta and lambda bookkeeping in double.
// kAlignSign (Jacobi sweeps): x <- -y / ||y|| when <y, x> < 0, so the new
// vector keeps the old one's orientation.
template <typename Acc>
__global__ __launch_bounds__(kNormBlock) void k_normalize(const Acc* y, i64 n, double* x, Acc* wv,
                                                          hopm_stats* st, int flags,
                                                          double* norm_out) {
  __shared__ double sh[kNormBlock / kWave];
  double ss = 0.0, yx = 0.0;
  for (i64 i = threadIdx.x; i < n; i += kNormBlock) {
    const double v = (double)y[i];
    ss += v * v;
    yx += v * x[i];
  }
  ss = block_sum_1024(ss, sh);
  if (flags & kAlignSign) yx = block_sum_1024(yx, sh);
  const double nrm = sqrt(ss);
  if (norm_out && threadIdx.x == 0) *norm_out = nrm;
  if (!(nrm > 0.0) || !isfinite(nrm)) {
    if (threadIdx.x == 0) {
      st->status = TVC_EDEGENERATE;
      if (flags & kFirstJ) st->delta = 0.0;
      if (flags & kLastJ) {
        st->lambda = nrm;
        st->sweeps += 1;
      }
    }
    return;
  }
  const double inv = ((flags & kAlignSign) && yx < 0.0) ? -1.0 / nrm : 1.0 / nrm;
  double dd = 0.0;
  for (i64 i = threadIdx.x; i < n; i += kNormBlock) {
    const double v = (double)y[i] * inv;
    const double d = v - x[i];
    dd += d * d;
    x[i] = v;
    wv[i] = (Acc)v;
  }
  dd = block_sum_1024(dd, sh);
  if (threadIdx.x == 0) {
    const double dj = sqrt(dd);
    st->delta = (flags & kFirstJ) ? dj : fmax(st->delta, dj);
    if (flags & kLastJ) {
      st->lambda = nrm;
      st->sweeps += 1;
    }
  }
}

// w[r] = prod_{m} v_m[i_m(r)] over the modes given by (offs, dims), the
// last mode varying fastest; product formed in double, rounded once.
struct KronArgs {
  int nm;
  i64 dims[TVC_MAX_ORDER];
  i64 offs[TVC_MAX_ORDER];
};

template <typename Acc>
__global__ void k_kron(const double* x, KronArgs k, Acc* w, i64 n, const float* scale0, i64 sdiv) {
  for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (i64)gridDim.x * blockDim.x) {
    i64 rem = r;
    double p = 1.0;
    for (int m = k.nm - 1; m >= 0; --m) {
      i64 q, i;
      divmod(rem, k.dims[m], q, i);
      rem = q;
      p *= x[k.offs[m] + i];
    }
    if (scale0) {
      i64 q, i;
      divmod(r, sdiv, q, i);
      p *= (double)scale0[q];
    }
    w[r] = (Acc)p;
  }
}

// Large weight vectors: the product over the trailing modes whose extents
// multiply to B <= kKronLo values is formed once per workgroup in LDS, and a
// workgroup then writes whole chunks of B consecutive weights, each the
// LDS values times the chunk's product over the leading modes (one index
// split per chunk instead of one per mode per weight).  Products are formed
// in FP64 and rounded once.
constexpr int kKronLo = 4096;

template <typename Acc>
__global__ __launch_bounds__(256) void k_kron_chunked(const double* x, KronArgs k, int h, i64 B, Acc* w,
                                                      i64 n) {
  __shared__ double lo[kKronLo];
  // The table one mode at a time, last mode first (its index varies
  // fastest): entries i * len + j of the next table are entry j of the
  // current one times x_m[i], the same products in the same order as one
  // mode after another per entry.  In place: i >= 1 first, then i = 0.
  if (threadIdx.x == 0) lo[0] = 1.0;
  __syncthreads();
  int len = 1;
  for (int m = k.nm - 1; m >= k.nm - h; --m) {
    const double* xm = x + k.offs[m];
    const int dm = (int)k.dims[m];
    for (int t = threadIdx.x; t < (dm - 1) * len; t += blockDim.x) {
      const int i = 1 + t / len, j = t % len;
      lo[i * len + j] = lo[j] * xm[i];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < len; j += blockDim.x) lo[j] *= xm[0];
    __syncthreads();
    len *= dm;
  }
  const i64 nchunks = n / B;
  for (i64 c = blockIdx.x; c < nchunks; c += gridDim.x) {
    i64 rem = c;
    double hi = 1.0;
    for (int m = k.nm - h - 1; m >= 0; --m) {
      i64 q, i;
      divmod(rem, k.dims[m], q, i);
      rem = q;
      hi *= x[k.offs[m] + i];
    }
    Acc* dst = w + c * B;
    for (i64 j = threadIdx.x; j < B; j += blockDim.x) dst[j] = (Acc)(hi * lo[j]);
  }
}

// ---------------------------------------------------------------- small steps
// The vector side of a sweep, once its operands are small (the n0 x n1
// matrix, the W chain below 64K values), as a short program that one
// workgroup runs instead of one launch per step: contract the last or the
// first mode of a buffer with a vector mirror, normalise into x_j with the
// sweep's bookkeeping (as k_normalize), and form the pass-2 weights
// x_0 (x) x_1, or copy every x into its mirror (the end of a Jacobi
// sweep).  Buffers 0..2 are LDS (kTailElems values each), the others
// global.
// Steps are separated by workgroup barriers, so a step sees the vectors the
// previous normalisations wrote.
constexpr int kTailThreads = 512;
constexpr int kTailElems = 2048;
constexpr int kTailMaxSteps = 48;
constexpr int kTailLds = 3;
constexpr int kTailGlobal = 12;
enum TailOp { kTLast = 0, kTFirst = 1, kTNorm = 2, kTKron = 3, kTCopy = 4, kTMirror = 5 };

struct TailStep {
  int op, src, dst, mode, flags;
  i64 a, b;   // kTLast: rows, n; kTFirst: n, rest; kTNorm: n; kTKron: n0, n1; kTCopy: n
};
static_assert(kTailMaxSteps * sizeof(TailStep) + 1024 < 4096, "small-step program exceeds the kernel argument space");

template <typename Acc>
struct TailProg {
  int nsteps;
  TailStep st[kTailMaxSteps];
  Acc* g[kTailGlobal];       // global buffers kTailLds ...
  double* x;
  Acc* wv;
  hopm_stats* stats;
  double* norms;             // optional: ||y|| of step j written to norms[j]
  const float* scale0;       // kTKron: optional per-row scale (E4M3 slabs)
  i64 sdiv;
  int d;
  i64 n[TVC_MAX_ORDER], off[TVC_MAX_ORDER], woff[TVC_MAX_ORDER];
};

template <typename Acc>
__device__ __forceinline__ double tail_block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < kTailThreads / kWave; ++q) t += sh[q];
  __syncthreads();
  return t;
}

template <typename Acc>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailProg<Acc> p) {
  __shared__ Acc lds[kTailLds][kTailElems];
  __shared__ double sh[kTailThreads / kWave];
  const int tid = threadIdx.x;
  for (int k = 0; k < p.nsteps; ++k) {
    const TailStep& q = p.st[k];
    const Acc* in = nullptr;
    if (q.src >= 0) in = q.src < kTailLds ? lds[q.src] : p.g[q.src - kTailLds];
    Acc* out = nullptr;
    if (q.dst >= 0) out = q.dst < kTailLds ? lds[q.dst] : p.g[q.dst - kTailLds];
    if (q.op == kTLast) {
      // out[r] = sum_i in[r * n + i] * w[i]; G lanes per row
      const i64 rows = q.a, n = q.b;
      const Acc* w = p.wv + p.woff[q.mode];
      // G lanes per row: up to the row's length (at most a wave), but no
      // more than lets every row into one pass of the workgroup where that
      // leaves at least 8 (a pass waits for its loads; in global memory
      // that is a round trip per pass)
      int G = 1;
      while (G < kWave && G < n) G <<= 1;
      while (G > 8 && (i64)(kTailThreads / G) < rows) G >>= 1;
      const int sub = tid & (G - 1);
      const int grp = tid / G, ngrp = kTailThreads / G;
      for (i64 r0 = 0; r0 < rows; r0 += ngrp) {
        const i64 r = r0 + grp;
        Acc acc = (Acc)0;
        if (r < rows) {
          const Acc* row = in + r * n;
          i64 i = sub;
          for (; i + 3 * G < n; i += 4 * G) {   // four loads issued, then summed in order
            const Acc v0 = row[i], v1 = row[i + G], v2 = row[i + 2 * G], v3 = row[i + 3 * G];
            const Acc w0 = w[i], w1 = w[i + G], w2 = w[i + 2 * G], w3 = w[i + 3 * G];
            acc = fma(v0, w0, acc);
            acc = fma(v1, w1, acc);
            acc = fma(v2, w2, acc);
            acc = fma(v3, w3, acc);
          }
          for (; i < n; i += G) acc = fma(row[i], w[i], acc);
        }
        for (int o = G >> 1; o >= 1; o >>= 1) acc += shfl_xor(acc, o);
        if (sub == 0 && r < rows) out[r] = acc;
      }
    } else if (q.op == kTFirst) {
      // out[c] = sum_i in[i * rest + c] * w[i]
      const i64 n = q.a, rest = q.b;
      const Acc* w = p.wv + p.woff[q.mode];
      for (i64 c = tid; c < rest; c += kTailThreads) {
        Acc acc = (Acc)0;
        i64 i = 0;
        for (; i + 8 <= n; i += 8) {   // eight loads issued, then summed in order
          Acc v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = in[(i + u) * rest + c];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc = fma(v[u], w[i + u], acc);
        }
        for (; i < n; ++i) acc = fma(in[i * rest + c], w[i], acc);
        out[c] = acc;
      }
    } else if (q.op == kTNorm) {
      const i64 n = q.a;
      const int j = q.mode;
      double* x = p.x + p.off[j];
      Acc* wj = p.wv + p.woff[j];
      double ss = 0.0, yx = 0.0;
      for (i64 i = tid; i < n; i += kTailThreads) {
        const double v = (double)in[i];
        ss += v * v;
        yx += v * x[i];
      }
      ss = tail_block_sum<Acc>(ss, sh);
      if (q.flags & kAlignSign) yx = tail_block_sum<Acc>(yx, sh);
      const double nrm = sqrt(ss);
      if (p.norms && tid == 0) p.norms[j] = nrm;
      if (!(nrm > 0.0) || !isfinite(nrm)) {
        if (tid == 0) {
          p.stats->status = TVC_EDEGENERATE;
          if (q.flags & kFirstJ) p.stats->delta = 0.0;
          if (q.flags & kLastJ) {
            p.stats->lambda = nrm;
            p.stats->sweeps += 1;
          }
        }
      } else {
        const double inv = ((q.flags & kAlignSign) && yx < 0.0) ? -1.0 / nrm : 1.0 / nrm;
        double dd = 0.0;
        for (i64 i = tid; i < n; i += kTailThreads) {
          const double v = (double)in[i] * inv;
          const double df = v - x[i];
          dd += df * df;
          x[i] = v;
          if (!(q.flags & kNoMirror)) wj[i] = (Acc)v;
        }
        dd = tail_block_sum<Acc>(dd, sh);
        if (tid == 0) {
          const double dj = sqrt(dd);
          p.stats->delta = (q.flags & kFirstJ) ? dj : fmax(p.stats->delta, dj);
          if (q.flags & kLastJ) {
            p.stats->lambda = nrm;
            p.stats->sweeps += 1;
          }
        }
      }
    } else if (q.op == kTCopy) {
      for (i64 i = tid; i < q.a; i += kTailThreads) out[i] = in[i];
    } else if (q.op == kTMirror) {
      for (int j = 0; j < p.d; ++j)
        for (i64 i = tid; i < p.n[j]; i += kTailThreads) p.wv[p.woff[j] + i] = (Acc)p.x[p.off[j] + i];
    } else {  // kTKron: out[r] = x_0[r / n1] * x_1[r mod n1] (* scale0[r / sdiv])
      const i64 n0 = q.a, n1 = q.b;
      const double* x0 = p.x + p.off[0];
      const double* x1 = p.x + p.off[1];
      for (i64 r = tid; r < n0 * n1; r += kTailThreads) {
        i64 i0, i1;
        divmod(r, n1, i0, i1);
        double v = x1[i1] * x0[i0];
        if (p.scale0) {
          i64 sq, sr;
          divmod(r, p.sdiv, sq, sr);
          v *= (double)p.scale0[sq];
        }
        out[r] = (Acc)v;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- schedule
namespace {

struct Layout {
  int dt = TVC_F32;
  int acc_dt = TVC_F32;       // dtype naming the accumulation type
  size_t ab = 4;
  int d = 0;
  i64 n[TVC_MAX_ORDER] = {};
  i64 off[TVC_MAX_ORDER] = {};   // offsets of the double vectors in x
  i64 woff[TVC_MAX_ORDER] = {};  // offsets of their mirrors in wv (16-byte aligned)
  i64 wsum = 0;
  i64 nsum = 0, nmax = 0, N = 0, R1 = 1, n01 = 1;
  // byte offsets into ws
  size_t o_wv = 0, o_y = 0, o_M = 0, o_w1 = 0, o_w2 = 0, o_Wa = 0, o_Ca = 0, o_Cb = 0,
         o_stats = 0, o_part = 0, o_Y = 0, o_J = 0, o_uv = 0, o_L = 0, o_dpart = 0;
  size_t part_bytes = 0, dpart_bytes = 0;
  size_t total = 0;
};

// Inputs in global memory up to this many values are read by the single
// workgroup of a small-step program (about 32 KB in float32: a few
// microseconds); larger ones get a full launch.
constexpr i64 kTailIn = 8192;

// Both sweeps take the vectors of the modes of W = A x_0 x_0 x_1 x_1
// (modes 2..d-1 kept) by halving: a node holding modes [a, b) of more than
// kTailIn values is read as the matrix [modes a..a+s)][modes a+s..b),
// s = (b - a) / 2, giving its contractions over the second half (the
// first-half node) and over the first half (the second-half node): in one
// pass for a Jacobi sweep, in two for a Gauss-Seidel sweep, whose second
// contraction takes the first half's new vectors; nodes of at most kTailIn
// values go to the small-step program.  Every node's
// two outputs get their own stretch of the split buffer (a pending
// small-step program may still read an earlier one), taken in the order the
// sweep visits the nodes.  f(a, s, b, P, Q, mo, zo) per split: P x Q the
// matrix, mo / zo the value offsets of its outputs.
inline i64 split_pad(i64 v) { return (v + 63) / 64 * 64; }

template <typename F>
void jacobi_splits(const i64* n, int a, int b, i64 size, i64& top, F&& f) {
  if (b - a <= 1 || size <= kTailIn) return;
  const int s = (b - a) / 2;
  i64 P = 1;
  for (int k = a; k < a + s; ++k) P *= n[k];
  const i64 Q = size / P;
  const i64 mo = top, zo = top + split_pad(P);
  top = zo + split_pad(Q);
  f(a, s, b, P, Q, mo, zo);
  jacobi_splits(n, a, a + s, P, top, f);
  jacobi_splits(n, a + s, b, Q, top, f);
}

// Every contraction a sweep performs, as (dtype, L, M, R); the workspace
// must hold the largest partial-sum scratch among them.
void sweep_tvcs(const Layout& Lt, std::vector<std::array<i64, 4>>& out) {
  const int d = Lt.d;
  const i64* n = Lt.n;
  if (d == 2) {
    out.push_back({Lt.dt, n[0], n[1], 1});
    out.push_back({Lt.dt, 1, n[0], n[1]});
    return;
  }
  out.push_back({Lt.dt, Lt.n01, Lt.R1, 1});            // pass 1
  out.push_back({Lt.acc_dt, n[0], n[1], 1});           // M x_1
  out.push_back({Lt.acc_dt, 1, n[0], n[1]});           // M^T x_0
  out.push_back({Lt.dt, 1, Lt.n01, Lt.R1});            // pass 2
  // the halving of W_2 (rows, then columns, of each node above kTailIn
  // values); the one-pass kernel of Jacobi sweeps sizes its own scratch
  i64 top = 0;
  if (d >= 4)
    jacobi_splits(n, 2, d, Lt.R1, top, [&](int, int, int, i64 P, i64 Q, i64, i64) {
      out.push_back({Lt.acc_dt, P, Q, 1});
      out.push_back({Lt.acc_dt, 1, P, Q});
    });
  // the leave-one-out chains on W_2 of hopm_leave_one_out: each contracts
  // modes k = d-1 .. 2 except the kept mode m
  for (int m = 2; m < d; ++m) {
    i64 left = Lt.R1, right = 1;   // left: modes before k still present
    for (int k = d - 1; k >= 2; --k) {
      left /= n[k];
      if (k == m) {
        right = n[k];
        continue;
      }
      out.push_back({Lt.acc_dt, left, n[k], right});
    }
  }
}

Layout make_layout(const tvc_tensor* A) {
  Layout Lt;
  Lt.dt = A->dtype;
  Lt.acc_dt = A->dtype == TVC_F64 ? TVC_F64 : TVC_F32;
  Lt.ab = acc_bytes(A->dtype);
  Lt.d = A->order;
  Lt.N = 1;
  const i64 per16 = 16 / (i64)acc_bytes(A->dtype);
  for (int i = 0; i < Lt.d; ++i) {
    Lt.n[i] = A->dims[i];
    Lt.off[i] = Lt.nsum;
    Lt.nsum += Lt.n[i];
    Lt.woff[i] = Lt.wsum;
    Lt.wsum += (Lt.n[i] + per16 - 1) / per16 * per16;
    Lt.nmax = std::max(Lt.nmax, Lt.n[i]);
    Lt.N *= Lt.n[i];
  }
  if (Lt.d >= 3) {
    Lt.n01 = Lt.n[0] * Lt.n[1];
    Lt.R1 = Lt.N / Lt.n01;
  }
  const size_t ab = Lt.ab;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  Lt.o_stats = take(sizeof(hopm_stats));
  Lt.o_wv = take((size_t)Lt.wsum * ab);
  Lt.o_y = take((size_t)Lt.nmax * ab);
  if (Lt.d >= 3) {
    Lt.o_M = take((size_t)Lt.n01 * ab);
    Lt.o_w2 = take((size_t)Lt.n01 * ab);
    Lt.o_w1 = take(Lt.d >= 4 ? (size_t)Lt.R1 * ab : 0);
    Lt.o_Wa = take((size_t)Lt.R1 * ab);
    i64 nmin = Lt.R1;
    for (int k = 2; k < Lt.d; ++k) nmin = std::min(nmin, Lt.n[k]);
    const size_t c = Lt.d >= 4 ? (size_t)(Lt.R1 / nmin) * ab : 0;
    Lt.o_Ca = take(c);
    Lt.o_Cb = take(c);
  } else {
    Lt.o_w2 = take((size_t)Lt.n[0] * ab);   // scaled weights for E4M3 (d = 2)
  }
  std::vector<std::array<i64, 4>> tv;
  sweep_tvcs(Lt, tv);
  size_t pb = 0;
  for (auto& t : tv)
    for (int a16 = 0; a16 < 2; ++a16)
      for (int w16 = 0; w16 < 2; ++w16)
        pb = std::max(pb, plan_tvc((int)t[0], t[1], t[2], t[3], a16, w16).part_bytes);
  Lt.part_bytes = pb;
  Lt.o_part = take(pb);
  // Jacobi sweeps: the d contraction results; both sweeps: the outputs and
  // the Kronecker weights of the halving of W; the one-pass scratch
  Lt.o_Y = take((size_t)Lt.wsum * ab);
  i64 jtop = 0, uvmax = 0;
  size_t jpart = 0;
  if (Lt.d >= 4)
    jacobi_splits(Lt.n, 2, Lt.d, Lt.R1, jtop, [&](int, int, int, i64 P, i64 Q, i64, i64) {
      for (int a4 = 0; a4 < 2; ++a4) jpart = std::max(jpart, plan_dual(Lt.acc_dt, P, Q, a4).part_bytes);
      uvmax = std::max(uvmax, split_pad(P) + Q);   // the two halves' Kronecker weights
    });
  Lt.o_J = take((size_t)jtop * ab);
  Lt.o_uv = take((size_t)uvmax * ab);
  // the leaves' global buffers of a Gauss-Seidel sweep
  Lt.o_L = take(Lt.d >= 3 ? (size_t)(3 * kTailIn) * ab : 0);
  const i64 P = Lt.d >= 3 ? Lt.n01 : Lt.n[0];
  const i64 R = Lt.d >= 3 ? Lt.R1 : (Lt.d == 2 ? Lt.n[1] : 1);
  // the one-pass scratch also serves pass 1 as strips (rows only)
  Lt.dpart_bytes = 0;
  for (int a4 = 0; a4 < 2; ++a4)
    for (int cols = 0; cols < 2; ++cols)
      Lt.dpart_bytes = std::max(Lt.dpart_bytes, plan_dual(Lt.dt, P, R, a4, cols).part_bytes);
  Lt.dpart_bytes = std::max(Lt.dpart_bytes, jpart);
  Lt.o_dpart = take(Lt.dpart_bytes);
  Lt.total = o;
  return Lt;
}

struct Ctx {
  const Layout* Lt;
  const tvc_tensor* A;
  double* x;
  char* ws;
  hopm_stats* st;
  hipStream_t s;
  double* norms = nullptr;   // optional: ||y|| of every (sweep, j) step
  template <typename P> P* at(size_t o) const { return (P*)(ws + o); }
};

#define TVC_TRY_HIP(expr)                                                                 \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(TVC_EHIP, std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

tvc_status run(const Ctx& c, int dt, const void* A, i64 L, i64 M, i64 R, const void* w, void* y,
               const float* oscale, i64 odiv) {
  return tvc_run_auto(dt, A, L, M, R, w, y, 1.0, 0.0, oscale, odiv, c.ws + c.Lt->o_part,
                      c.Lt->part_bytes, c.s, kRoleHopm);
}

template <typename Acc>
tvc_status normalize(const Ctx& c, const void* y, int j, int extra_flags = 0) {
  const Layout& Lt = *c.Lt;
  int flags = (j == 0 ? kFirstJ : 0) | (j == Lt.d - 1 ? kLastJ : 0) | extra_flags;
  hipLaunchKernelGGL((k_normalize<Acc>), dim3(1), dim3(kNormBlock), 0, c.s, (const Acc*)y,
                     Lt.n[j], c.x + Lt.off[j], c.at<Acc>(Lt.o_wv) + Lt.woff[j], c.st, flags,
                     c.norms ? c.norms + j : nullptr);
  TVC_TRY_HIP(hipGetLastError());
  return TVC_OK;
}

template <typename Acc>
tvc_status kron(const Ctx& c, int m0, int m1, Acc* w, const float* scale0, i64 sdiv) {
  const Layout& Lt = *c.Lt;
  KronArgs k;
  k.nm = m1 - m0;
  i64 n = 1;
  for (int m = m0; m < m1; ++m) {
    k.dims[m - m0] = Lt.n[m];
    k.offs[m - m0] = Lt.off[m];
    n *= Lt.n[m];
  }
  // trailing modes whose product fits the LDS table
  int h = 0;
  i64 B = 1;
  while (h < k.nm && B * k.dims[k.nm - 1 - h] <= kKronLo) B *= k.dims[k.nm - 1 - h++];
  if (!scale0 && n >= ((i64)1 << 16) && B >= 64) {
    const int g = (int)std::max<i64>(1, std::min<i64>(n / B, 4 * (i64)device_cus()));
    hipLaunchKernelGGL((k_kron_chunked<Acc>), dim3(g), dim3(256), 0, c.s, (const double*)c.x, k, h, B,
                       w, n);
  } else {
    const int g = (int)std::max<i64>(1, std::min<i64>((n + 255) / 256, 4 * (i64)device_cus()));
    hipLaunchKernelGGL((k_kron<Acc>), dim3(g), dim3(256), 0, c.s, (const double*)c.x, k, w, n, scale0,
                       sdiv);
  }
  TVC_TRY_HIP(hipGetLastError());
  return TVC_OK;
}

#define TVC_TRY(expr)                 \
  do {                                \
    tvc_status s_ = (expr);           \
    if (s_ != TVC_OK) return s_;      \
  } while (0)

// A buffer of a small-step program: LDS slot 0..2 or a global pointer.
template <typename Acc>
struct TBufT {
  int lds_id = -1;
  Acc* ptr = nullptr;
  i64 size = 0;
  static TBufT lds(int id, i64 n) { TBufT b; b.lds_id = id; b.size = n; return b; }
  static TBufT global(Acc* p, i64 n) { TBufT b; b.ptr = p; b.size = n; return b; }
  bool is_global() const { return lds_id < 0; }
};

// An LDS slot holding neither a nor b.
template <typename B>
int tl_free_lds(const B& a, const B& b) {
  for (int i = 0; i < kTailLds; ++i)
    if (i != a.lds_id && i != b.lds_id) return i;
  return 0;
}

// Collects small steps and launches them as one k_tail program.
template <typename Acc>
struct Tail {
  typedef TBufT<Acc> TBuf;
  const Ctx& c;
  TailProg<Acc> p{};
  int nglob = 0;

  explicit Tail(const Ctx& cc) : c(cc) { reset(); }

  void reset() {
    const Layout& Lt = *c.Lt;
    p = TailProg<Acc>{};
    p.x = c.x;
    p.wv = c.at<Acc>(Lt.o_wv);
    p.stats = c.st;
    p.norms = c.norms;
    p.sdiv = 1;
    p.d = Lt.d;
    for (int m = 0; m < Lt.d; ++m) {
      p.n[m] = Lt.n[m];
      p.off[m] = Lt.off[m];
      p.woff[m] = Lt.woff[m];
    }
    nglob = 0;
  }

  tvc_status flush() {
    if (p.nsteps == 0) return TVC_OK;
    hipLaunchKernelGGL((k_tail<Acc>), dim3(1), dim3(kTailThreads), 0, c.s, p);
    TVC_TRY_HIP(hipGetLastError());
    reset();
    return TVC_OK;
  }

  // buffer id for the program (registering a global pointer); flushes when
  // the program is full
  tvc_status id(const TBuf& b, int* out) {
    if (!b.is_global()) {
      *out = b.lds_id;
      return TVC_OK;
    }
    for (int i = 0; i < nglob; ++i)
      if (p.g[i] == b.ptr) {
        *out = kTailLds + i;
        return TVC_OK;
      }
    if (nglob == (int)(sizeof(p.g) / sizeof(p.g[0]))) return fail(TVC_EINVAL, "small-step program: too many buffers");
    p.g[nglob] = b.ptr;
    *out = kTailLds + nglob++;
    return TVC_OK;
  }

  tvc_status add(int op, const TBuf* src, const TBuf* dst, int mode, int flags, i64 a, i64 b) {
    if (p.nsteps == kTailMaxSteps) return fail(TVC_EINVAL, "small-step program: too many steps");
    TailStep q{};
    q.op = op;
    q.mode = mode;
    q.flags = flags;
    q.a = a;
    q.b = b;
    q.src = -1;
    q.dst = -1;
    if (src) TVC_TRY(id(*src, &q.src));
    if (dst) TVC_TRY(id(*dst, &q.dst));
    p.st[p.nsteps++] = q;
    return TVC_OK;
  }

  tvc_status last(const TBuf& src, i64 rows, i64 n, int mode, const TBuf& dst) {
    return add(kTLast, &src, &dst, mode, 0, rows, n);
  }
  tvc_status first(const TBuf& src, i64 n, i64 rest, int mode, const TBuf& dst) {
    return add(kTFirst, &src, &dst, mode, 0, n, rest);
  }
  tvc_status norm(const TBuf& src, int j, int extra_flags = 0) {
    const Layout& Lt = *c.Lt;
    const int flags = (j == 0 ? kFirstJ : 0) | (j == Lt.d - 1 ? kLastJ : 0) | extra_flags;
    return add(kTNorm, &src, nullptr, j, flags, Lt.n[j], 0);
  }
  tvc_status mirror() { return add(kTMirror, nullptr, nullptr, 0, 0, 0, 0); }
  tvc_status copy(const TBuf& src, const TBuf& dst) {
    return add(kTCopy, &src, &dst, 0, 0, src.size, 0);
  }
  int room() const { return kTailMaxSteps - p.nsteps; }
  tvc_status kron(const TBuf& dst, i64 n0, i64 n1, const float* scale0, i64 sdiv) {
    p.scale0 = scale0;
    p.sdiv = sdiv;
    return add(kTKron, nullptr, &dst, 0, 0, n0, n1);
  }
};

// Pass 1 of a sweep contracts the n_0 n_1 rows of A with the Kronecker
// weights x_2 (x) ... (x) x_{d-1}.  As strips (run_dual without the column
// sums) each wave keeps the weights of its columns in registers for a whole
// chunk of rows; the row kernel re-reads them per row group instead.  With
// rows of 2^17 elements and more (512 KB or more of weights) the strips are
// faster in the 4-byte and narrower formats (measured: 32^6 sweep bf16 0.729
// -> 0.702 ms, E4M3 0.491 -> 0.407, 63^5 float32 1.61 -> 1.51, 8^10 1.53 ->
// 1.48; float32 32^6 and 10^9 unchanged); on shorter rows the row kernel is
// (175^4: 1.30 against 1.39).  float64 rows, which preload their next step,
// are faster than the strips (63^5 sweep 2.61 against 3.26 ms).
bool pass1_strips(const Ctx& c) {
  const int t = tuning().strip_rows;
  if (t != 0) return t > 0;
  return c.A->dtype != TVC_F64 && c.Lt->R1 >= ((i64)1 << 17) && c.Lt->n01 >= 16;
}

template <typename Acc>
tvc_status sweep(const Ctx& c) {
  const Layout& Lt = *c.Lt;
  const tvc_tensor* A = c.A;
  const int d = Lt.d;
  const i64* n = Lt.n;
  Acc* wv = c.at<Acc>(Lt.o_wv);
  Acc* y = c.at<Acc>(Lt.o_y);
  const bool f8 = A->dtype == TVC_F8E4M3;
  if (d == 2) {
    TVC_TRY(run(c, A->dtype, A->data, n[0], n[1], 1, wv + Lt.woff[1], y,
                f8 ? A->slab_scale : nullptr, 1));
    TVC_TRY(normalize<Acc>(c, y, 0));
    const Acc* w0 = wv + Lt.woff[0];
    if (f8) {
      Acc* sw = c.at<Acc>(Lt.o_w2);
      TVC_TRY(kron<Acc>(c, 0, 1, sw, A->slab_scale, 1));
      w0 = sw;
    }
    TVC_TRY(run(c, A->dtype, A->data, 1, n[0], n[1], w0, y, nullptr, 1));
    return normalize<Acc>(c, y, 1);
  }
  Acc* Mm = c.at<Acc>(Lt.o_M);
  Acc* w2 = c.at<Acc>(Lt.o_w2);
  Acc* Wa = c.at<Acc>(Lt.o_Wa);
  typedef TBufT<Acc> TBuf;
  Tail<Acc> tl(c);
  // pass 1: M = A contracted over modes 2..d-1
  const Acc* w1 = wv + Lt.woff[2];
  if (d >= 4) {
    Acc* w1b = c.at<Acc>(Lt.o_w1);
    TVC_TRY(kron<Acc>(c, 2, d, w1b, nullptr, 1));
    w1 = w1b;
  }
  if (pass1_strips(c)) {
    const DualPlan p = plan_dual(A->dtype, Lt.n01, Lt.R1, ((uintptr_t)A->data % 4) == 0, false);
    TVC_TRY_HIP(run_dual(A->dtype, A->data, Lt.n01, Lt.R1, w1, nullptr, Mm, nullptr,
                         f8 ? A->slab_scale : nullptr, n[1], p, c.ws + Lt.o_dpart, c.s));
  } else {
    TVC_TRY(run(c, A->dtype, A->data, Lt.n01, Lt.R1, 1, w1, Mm, f8 ? A->slab_scale : nullptr, n[1]));
  }
  // j = 0, 1 and the pass-2 weights: one small program when M is small
  if (Lt.n01 <= kTailIn && n[0] <= kTailElems && n[1] <= kTailElems) {
    const TBuf m = TBuf::global(Mm, Lt.n01), l0 = TBuf::lds(0, n[0]), l1 = TBuf::lds(1, n[1]);
    TVC_TRY(tl.last(m, n[0], n[1], 1, l0));
    TVC_TRY(tl.norm(l0, 0));
    TVC_TRY(tl.first(m, n[0], n[1], 0, l1));
    TVC_TRY(tl.norm(l1, 1));
    TVC_TRY(tl.kron(TBuf::global(w2, Lt.n01), n[0], n[1], f8 ? A->slab_scale : nullptr, n[1]));
    TVC_TRY(tl.flush());
  } else {
    TVC_TRY(run(c, Lt.acc_dt, Mm, n[0], n[1], 1, wv + Lt.woff[1], y, nullptr, 1));
    TVC_TRY(normalize<Acc>(c, y, 0));
    TVC_TRY(run(c, Lt.acc_dt, Mm, 1, n[0], n[1], wv + Lt.woff[0], y, nullptr, 1));
    TVC_TRY(normalize<Acc>(c, y, 1));
    TVC_TRY(kron<Acc>(c, 0, 2, w2, f8 ? A->slab_scale : nullptr, n[1]));
  }
  // pass 2: W_2 = A contracted with x_0 (x) x_1 (slab scale folded into the weights)
  TVC_TRY(run(c, A->dtype, A->data, 1, Lt.n01, Lt.R1, w2, Wa, nullptr, 1));
  // j >= 2: the modes of W_2 in Gauss-Seidel order, by halving (see
  // jacobi_splits for the node layout).  A node T holding modes [a, b) and
  // more than kTailIn values is read as the matrix [modes a..h)[modes h..b):
  // its rows against the previous x_h..x_{b-1} give the node of the first
  // half, whose vectors are then updated in order; its columns against those
  // new x_a..x_{h-1} give the node of the second half.  Each x_j thus sees
  // the new vectors of the modes before it and the previous ones of the
  // modes after it, as in the chain of Algorithm 1, and W_2 is read twice per
  // level instead of once per kept mode.  Nodes of at most kTailIn values
  // run the chain in the small-step program.
  Acc* J = c.at<Acc>(Lt.o_J);
  Acc* uv = c.at<Acc>(Lt.o_uv);
  Acc* const Lb[3] = {c.at<Acc>(Lt.o_L), c.at<Acc>(Lt.o_L) + kTailIn, c.at<Acc>(Lt.o_L) + 2 * kTailIn};
  // a leaf buffer holding neither x1 nor x2
  auto lfree = [&](const TBuf& x1, const TBuf& x2) -> Acc* {
    for (Acc* q : Lb)
      if (!(x1.is_global() && x1.ptr == q) && !(x2.is_global() && x2.ptr == q)) return q;
    return Lb[0];
  };
  auto leaf = [&](const TBuf& T, int a, int b) -> tvc_status {
    TBuf W = T;
    for (int j = a; j < b; ++j) {
      // j's steps (at most one contraction of W, b - 1 - j of the chain and
      // the normalisation) pass values through LDS, so they share a program;
      // W moves to a global buffer first when the pending one must be run.
      if (tl.room() < (j > a ? 1 : 0) + (b - 1 - j) + 1 + 1) {   // + 1: the copy of W
        if (!W.is_global()) {
          const TBuf dst = TBuf::global(lfree(W, W), W.size);
          TVC_TRY(tl.copy(W, dst));
          W = dst;
        }
        TVC_TRY(tl.flush());
      }
      if (j > a) {   // W_j = W_{j-1} contracted over its first mode (j - 1), new x_{j-1}
        const i64 out = W.size / n[j - 1];
        const TBuf dst = out <= kTailElems ? TBuf::lds(tl_free_lds(W, W), out)
                                           : TBuf::global(lfree(W, W), out);
        TVC_TRY(tl.first(W, n[j - 1], out, j - 1, dst));
        W = dst;
      }
      // y_j = W_j contracted over modes b-1 .. j+1 (previous vectors)
      TBuf src = W;
      i64 t = W.size;
      for (int m = b - 1; m > j; --m) {
        const i64 out = t / n[m];
        const TBuf dst = out <= kTailElems ? TBuf::lds(tl_free_lds(W, src), out)
                                           : TBuf::global(lfree(W, src), out);
        TVC_TRY(tl.last(src, out, n[m], m, dst));
        src = dst;
        t = out;
      }
      TVC_TRY(tl.norm(src, j));
    }
    return TVC_OK;
  };
  i64 top = 0;
  std::function<tvc_status(const TBuf&, int, int)> node = [&](const TBuf& T, int a, int b) -> tvc_status {
    if (b - a <= 1 || T.size <= kTailIn) return leaf(T, a, b);
    const int h = a + (b - a) / 2;
    i64 P = 1;
    for (int k = a; k < h; ++k) P *= n[k];
    const i64 Q = T.size / P;
    Acc* vo = J + top;
    Acc* uo = J + top + split_pad(P);
    top += split_pad(P) + split_pad(Q);
    // first half: rows against the previous x_h..x_{b-1} (no pending step
    // has changed them)
    TVC_TRY(kron<Acc>(c, h, b, uv + split_pad(P), nullptr, 1));
    TVC_TRY(run(c, Lt.acc_dt, T.ptr, P, Q, 1, uv + split_pad(P), vo, nullptr, 1));
    TVC_TRY(node(TBuf::global(vo, P), a, h));
    // second half: columns against the new x_a..x_{h-1} (their program first)
    TVC_TRY(tl.flush());
    TVC_TRY(kron<Acc>(c, a, h, uv, nullptr, 1));
    TVC_TRY(run(c, Lt.acc_dt, T.ptr, 1, P, Q, uv, uo, nullptr, 1));
    return node(TBuf::global(uo, Q), h, b);
  };
  TVC_TRY(node(TBuf::global(Wa, Lt.R1), 2, d));
  return tl.flush();
}

// ---------------------------------------------------------------- Jacobi sweep
// Jacobi HOPM, a variant of the method (the paper's sweep is Gauss-Seidel):
// every x_j of a sweep is the normalised contraction of A with the vectors
// of the previous sweep.  All d contractions then come from ONE pass over A
// (run_dual on the [n_0 n_1][n_2 ... n_{d-1}] view): M = A x_2 .. x_{d-1}
// gives y_0 = M x_1 and y_1 = M^T x_0, W_2 = A x_0 x_1 gives y_j (j >= 2)
// contracted with the other previous vectors (W halved into one-pass reads
// down to small-step programs, see jacobi_splits).  Each result is
// normalised with the sign that keeps <x_j(new), x_j(old)> >= 0 (without
// it, even orders can flip the signs of all vectors every sweep, and delta
// would never fall; the directions are the same), into x only: the
// contractions read the previous vectors from the mirror, which the sweep's
// last step refreshes.  lambda = ||y_{d-1}|| and delta as in a
// Gauss-Seidel sweep.
template <typename Acc>
tvc_status jacobi_sweep(const Ctx& c) {
  const Layout& Lt = *c.Lt;
  const tvc_tensor* A = c.A;
  const int d = Lt.d;
  const i64* n = Lt.n;
  Acc* wv = c.at<Acc>(Lt.o_wv);
  Acc* Y = c.at<Acc>(Lt.o_Y);
  const bool f8 = A->dtype == TVC_F8E4M3;
  const bool a4 = ((uintptr_t)A->data % 4) == 0;
  const Acc* ysrc[TVC_MAX_ORDER];
  for (int j = 0; j < d; ++j) ysrc[j] = Y + Lt.woff[j];
  if (d == 2) {
    const Acc* u = wv + Lt.woff[0];
    if (f8) {   // the slab scale of row i0 folded into the column weights
      Acc* sw = c.at<Acc>(Lt.o_w2);
      TVC_TRY(kron<Acc>(c, 0, 1, sw, A->slab_scale, 1));
      u = sw;
    }
    const DualPlan p = plan_dual(A->dtype, n[0], n[1], a4);
    TVC_TRY_HIP(run_dual(A->dtype, A->data, n[0], n[1], wv + Lt.woff[1], u, Y + Lt.woff[0],
                         Y + Lt.woff[1], f8 ? A->slab_scale : nullptr, 1, p, c.ws + Lt.o_dpart, c.s));
    for (int j = 0; j < d; ++j) TVC_TRY(normalize<Acc>(c, ysrc[j], j, kAlignSign));
    return TVC_OK;
  }
  typedef TBufT<Acc> TBuf;
  const Acc* w1 = wv + Lt.woff[2];
  if (d >= 4) {
    Acc* w1b = c.at<Acc>(Lt.o_w1);
    TVC_TRY(kron<Acc>(c, 2, d, w1b, nullptr, 1));
    w1 = w1b;
  }
  Acc* w2 = c.at<Acc>(Lt.o_w2);
  TVC_TRY(kron<Acc>(c, 0, 2, w2, f8 ? A->slab_scale : nullptr, n[1]));
  Acc* Mm = c.at<Acc>(Lt.o_M);
  Acc* Wa = c.at<Acc>(Lt.o_Wa);
  const DualPlan p = plan_dual(A->dtype, Lt.n01, Lt.R1, a4);
  TVC_TRY_HIP(run_dual(A->dtype, A->data, Lt.n01, Lt.R1, w1, w2, Mm, Wa,
                       f8 ? A->slab_scale : nullptr, n[1], p, c.ws + Lt.o_dpart, c.s));
  // Every x_j is normalised as soon as its contraction exists, with the
  // mirror left alone (the remaining contractions read the previous
  // vectors from it) and copied over by the program's last step.
  constexpr int kJ = kAlignSign | kNoMirror;
  Tail<Acc> tl(c);
  if (Lt.n01 <= kTailIn && n[0] <= kTailElems && n[1] <= kTailElems) {
    const TBuf m = TBuf::global(Mm, Lt.n01), l0 = TBuf::lds(0, n[0]), l1 = TBuf::lds(1, n[1]);
    TVC_TRY(tl.last(m, n[0], n[1], 1, l0));
    TVC_TRY(tl.norm(l0, 0, kJ));
    TVC_TRY(tl.first(m, n[0], n[1], 0, l1));
    TVC_TRY(tl.norm(l1, 1, kJ));
  } else {
    TVC_TRY(run(c, Lt.acc_dt, Mm, n[0], n[1], 1, wv + Lt.woff[1], Y + Lt.woff[0], nullptr, 1));
    TVC_TRY(run(c, Lt.acc_dt, Mm, 1, n[0], n[1], wv + Lt.woff[0], Y + Lt.woff[1], nullptr, 1));
    TVC_TRY(tl.norm(TBuf::global(Y + Lt.woff[0], n[0]), 0, kJ));
    TVC_TRY(tl.norm(TBuf::global(Y + Lt.woff[1], n[1]), 1, kJ));
  }
  // The leave-one-out vectors of a node of at most kTailIn values (modes
  // [a, b)): for each kept mode j, contract the modes after j from the last
  // one down, then the modes before j from the first one up.
  Acc* Ca = c.at<Acc>(Lt.o_Ca);
  Acc* Cb = c.at<Acc>(Lt.o_Cb);
  auto leaf = [&](const TBuf& T, int a, int b) -> tvc_status {
    for (int j = a; j < b; ++j) {
      if (tl.room() < (b - a - 1) + 1 + 1) TVC_TRY(tl.flush());   // + 1: the mirror step
      TBuf src = T;
      i64 t = T.size;
      auto next = [&](i64 out) {
        if (out <= kTailElems) return TBuf::lds(tl_free_lds(src, src), out);
        return TBuf::global(src.is_global() && src.ptr == Ca ? Cb : Ca, out);
      };
      for (int m = b - 1; m > j; --m) {
        const i64 out = t / n[m];
        const TBuf dst = next(out);
        TVC_TRY(tl.last(src, out, n[m], m, dst));
        src = dst;
        t = out;
      }
      for (int m = a; m < j; ++m) {
        const i64 out = t / n[m];
        const TBuf dst = next(out);
        TVC_TRY(tl.first(src, n[m], out, m, dst));
        src = dst;
        t = out;
      }
      TVC_TRY(tl.norm(src, j, kJ));
    }
    return TVC_OK;
  };
  // Nodes above kTailIn values: one pass over the node as a matrix (the
  // halves' Kronecker weights from the previous vectors in x, which no
  // launch so far has changed: the pending program runs after), then the
  // two halves.  Same offsets as the workspace sizing.
  Acc* J = c.at<Acc>(Lt.o_J);
  Acc* uv = c.at<Acc>(Lt.o_uv);
  i64 top = 0;
  std::function<tvc_status(const TBuf&, int, int)> node = [&](const TBuf& T, int a, int b) -> tvc_status {
    if (b - a <= 1 || T.size <= kTailIn) return leaf(T, a, b);
    const int s2 = (b - a) / 2;
    i64 P = 1;
    for (int k = a; k < a + s2; ++k) P *= n[k];
    const i64 Q = T.size / P;
    Acc* mo = J + top;
    Acc* zo = J + top + split_pad(P);
    top += split_pad(P) + split_pad(Q);
    TVC_TRY(kron<Acc>(c, a, a + s2, uv, nullptr, 1));
    TVC_TRY(kron<Acc>(c, a + s2, b, uv + split_pad(P), nullptr, 1));
    const DualPlan q = plan_dual(Lt.acc_dt, P, Q, true);
    TVC_TRY_HIP(run_dual(Lt.acc_dt, T.ptr, P, Q, uv + split_pad(P), uv, mo, zo, nullptr, 1, q,
                         c.ws + Lt.o_dpart, c.s));
    TVC_TRY(node(TBuf::global(mo, P), a, a + s2));
    return node(TBuf::global(zo, Q), a + s2, b);
  };
  TVC_TRY(node(TBuf::global(Wa, Lt.R1), 2, d));
  TVC_TRY(tl.mirror());
  return tl.flush();
}

template <typename Acc>
tvc_status iterate(const Ctx& c, int sweeps, bool jacobi = false) {
  const Layout& Lt = *c.Lt;
  const int g = (int)std::max<i64>(1, std::min<i64>((Lt.nsum + 255) / 256, 64));
  VecOffsets vo;
  vo.d = Lt.d;
  for (int m = 0; m < Lt.d; ++m) {
    vo.n[m] = Lt.n[m];
    vo.off[m] = Lt.off[m];
    vo.woff[m] = Lt.woff[m];
  }
  hipLaunchKernelGGL((k_prepare<Acc>), dim3(g), dim3(256), 0, c.s, (const double*)c.x,
                     c.at<Acc>(Lt.o_wv), vo, c.st);
  TVC_TRY_HIP(hipGetLastError());
  Ctx ci = c;
  for (int i = 0; i < sweeps; ++i) {
    TVC_TRY(jacobi ? jacobi_sweep<Acc>(ci) : sweep<Acc>(ci));
    if (ci.norms) ci.norms += Lt.d;
  }
  return TVC_OK;
}

tvc_status check_hopm_args(const tvc_tensor* A, double* x, void* ws, size_t ws_bytes,
                           const Layout& Lt) {
  TVC_TRY(check_tensor(A, "A"));
  if (A->order < 2) return fail(TVC_EINVAL, "HOPM needs order >= 2");
  if (!x) return fail(TVC_EINVAL, "x is NULL");
  if ((uintptr_t)x % 8 != 0) return fail(TVC_EINVAL, "x not 8-byte aligned");
  if (!ws || (uintptr_t)ws % 256 != 0 || ws_bytes < Lt.total)
    return fail(TVC_EWORKSPACE, "HOPM workspace of " + std::to_string(Lt.total) +
                                    " bytes (256-byte aligned) required");
  const size_t abytes = (size_t)numel(A) * elem_bytes(A->dtype);
  const size_t xbytes = (size_t)Lt.nsum * 8;
  if (overlaps(x, xbytes, A->data, abytes) || overlaps(ws, ws_bytes, A->data, abytes) ||
      overlaps(ws, ws_bytes, x, xbytes))
    return fail(TVC_EALIAS, "x, workspace and A must not overlap");
  return TVC_OK;
}

tvc_status iterate_any(const tvc_tensor* A, double* x, int sweeps, void* ws, size_t ws_bytes,
                       hopm_stats* st, hipStream_t s, double* norms = nullptr, bool jacobi = false) {
  Layout Lt = make_layout(A);
  TVC_TRY(check_hopm_args(A, x, ws, ws_bytes, Lt));
  if (sweeps < 1) return fail(TVC_EINVAL, "sweeps must be >= 1");
  if (!st) return fail(TVC_EINVAL, "stats pointer is NULL");
  if (norms && (uintptr_t)norms % 8) return fail(TVC_EINVAL, "norms misaligned");
  Ctx c{&Lt, A, x, (char*)ws, st, s, norms};
  if (A->dtype == TVC_F64) return iterate<double>(c, sweeps, jacobi);
  return iterate<float>(c, sweeps, jacobi);
}

// ---------------------------------------------------------------- leave-one-out
template <typename Acc>
__global__ void k_to_double(const Acc* y, double* out, i64 n) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    out[i] = (double)y[i];
}

template <typename Acc>
tvc_status to_double(const Ctx& c, const Acc* y, int m, double* out) {
  const i64 n = c.Lt->n[m];
  const int g = (int)std::max<i64>(1, std::min<i64>((n + 255) / 256, 64));
  hipLaunchKernelGGL((k_to_double<Acc>), dim3(g), dim3(256), 0, c.s, y, out + c.Lt->off[m], n);
  TVC_TRY_HIP(hipGetLastError());
  return TVC_OK;
}

// out_m = A contracted with the vectors c.x over every mode but m, for every
// m in `mask`: pass 1 (M) serves modes 0 and 1, pass 2 (W_2) the others,
// each then a chain of small contractions of W_2 that keeps mode m.
template <typename Acc>
tvc_status leave_one_out(const Ctx& c, uint32_t mask, double* out) {
  const Layout& Lt = *c.Lt;
  const tvc_tensor* A = c.A;
  const int d = Lt.d;
  const i64* n = Lt.n;
  const bool f8 = A->dtype == TVC_F8E4M3;
  VecOffsets vo;
  vo.d = d;
  for (int m = 0; m < d; ++m) {
    vo.n[m] = n[m];
    vo.off[m] = Lt.off[m];
    vo.woff[m] = Lt.woff[m];
  }
  hipLaunchKernelGGL((k_prepare<Acc>), dim3(16), dim3(256), 0, c.s, (const double*)c.x,
                     c.at<Acc>(Lt.o_wv), vo, c.st);
  TVC_TRY_HIP(hipGetLastError());
  Acc* wv = c.at<Acc>(Lt.o_wv);
  Acc* y = c.at<Acc>(Lt.o_y);
  if (d == 2) {
    if (mask & 1u) {
      TVC_TRY(run(c, A->dtype, A->data, n[0], n[1], 1, wv + Lt.woff[1], y,
                  f8 ? A->slab_scale : nullptr, 1));
      TVC_TRY(to_double<Acc>(c, y, 0, out));
    }
    if (mask & 2u) {
      const Acc* w0 = wv + Lt.woff[0];
      if (f8) {
        Acc* sw = c.at<Acc>(Lt.o_w2);
        TVC_TRY(kron<Acc>(c, 0, 1, sw, A->slab_scale, 1));
        w0 = sw;
      }
      TVC_TRY(run(c, A->dtype, A->data, 1, n[0], n[1], w0, y, nullptr, 1));
      TVC_TRY(to_double<Acc>(c, y, 1, out));
    }
    return TVC_OK;
  }
  Acc* Mm = c.at<Acc>(Lt.o_M);
  if (mask & 3u) {
    const Acc* w1 = wv + Lt.woff[2];
    if (d >= 4) {
      Acc* w1b = c.at<Acc>(Lt.o_w1);
      TVC_TRY(kron<Acc>(c, 2, d, w1b, nullptr, 1));
      w1 = w1b;
    }
    TVC_TRY(run(c, A->dtype, A->data, Lt.n01, Lt.R1, 1, w1, Mm, f8 ? A->slab_scale : nullptr, n[1]));
    if (mask & 1u) {
      TVC_TRY(run(c, Lt.acc_dt, Mm, n[0], n[1], 1, wv + Lt.woff[1], y, nullptr, 1));
      TVC_TRY(to_double<Acc>(c, y, 0, out));
    }
    if (mask & 2u) {
      TVC_TRY(run(c, Lt.acc_dt, Mm, 1, n[0], n[1], wv + Lt.woff[0], y, nullptr, 1));
      TVC_TRY(to_double<Acc>(c, y, 1, out));
    }
  }
  if (mask & ~3u) {
    Acc* w2 = c.at<Acc>(Lt.o_w2);
    Acc* Wa = c.at<Acc>(Lt.o_Wa);
    TVC_TRY(kron<Acc>(c, 0, 2, w2, f8 ? A->slab_scale : nullptr, n[1]));
    TVC_TRY(run(c, A->dtype, A->data, 1, Lt.n01, Lt.R1, w2, Wa, nullptr, 1));
    for (int m = 2; m < d; ++m) {
      if (!(mask & (1u << m))) continue;
      const Acc* src = Wa;
      Acc* bufs[2] = {c.at<Acc>(Lt.o_Ca), c.at<Acc>(Lt.o_Cb)};
      int bi = 0;
      i64 left = Lt.R1, right = 1;
      for (int k = d - 1; k >= 2; --k) {
        left /= n[k];
        if (k == m) {
          right = n[k];
          continue;
        }
        TVC_TRY(run(c, Lt.acc_dt, src, left, n[k], right, wv + Lt.woff[k], bufs[bi], nullptr, 1));
        src = bufs[bi];
        bi ^= 1;
      }
      TVC_TRY(to_double<Acc>(c, src, m, out));
    }
  }
  return TVC_OK;
}

// ---------------------------------------------------------------- reverse pass
// One step s = (sweep i, mode j) of the reverse pass through Gauss-Seidel
// sweeps, in one workgroup:
//   state before the step: x_m = xs_{i+1}[m] for m < j, xs_i[m] for m > j
//   ybar = (xbar_j - x_j <x_j, xbar_j>) / ||y|| + seed * x_j,  x_j = xs_{i+1}[j]
//   vecs = state with ybar at mode j (the operand of the leave-one-out pass),
//   factor slot = the same vectors (one rank-1 term of dA), xbar_j = 0.
__global__ __launch_bounds__(kNormBlock) void k_step_adjoint(const double* xs_i, const double* xs_i1,
                                                             VecOffsets vo, int j, const double* norm,
                                                             double seed, double* xbar, double* vecs,
                                                             double* factor) {
  __shared__ double sh[kNormBlock / kWave];
  const i64 o = vo.off[j], n = vo.n[j];
  double dot = 0.0;
  for (i64 i = threadIdx.x; i < n; i += kNormBlock) dot += xs_i1[o + i] * xbar[o + i];
  dot = block_sum_1024(dot, sh);
  const double nrm = *norm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (i64 i = threadIdx.x; i < n; i += kNormBlock) {
    const double xj = xs_i1[o + i];
    const double yb = (xbar[o + i] - xj * dot) * inv + seed * xj;
    vecs[o + i] = yb;
    factor[o + i] = yb;
    xbar[o + i] = 0.0;
  }
  for (int m = 0; m < vo.d; ++m) {
    if (m == j) continue;
    const double* src = m < j ? xs_i1 : xs_i;
    for (i64 i = threadIdx.x; i < vo.n[m]; i += kNormBlock) {
      const double v = src[vo.off[m] + i];
      vecs[vo.off[m] + i] = v;
      factor[vo.off[m] + i] = v;
    }
  }
}

// xbar_m += lo_m for every m != j
__global__ void k_accumulate(double* xbar, const double* lo, VecOffsets vo, int j) {
  for (int m = 0; m < vo.d; ++m) {
    if (m == j) continue;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < vo.n[m];
         i += (i64)gridDim.x * blockDim.x)
      xbar[vo.off[m] + i] += lo[vo.off[m] + i];
  }
}

__global__ void k_copy_f64(const double* s, double* d, i64 n, double v, int fill) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    d[i] = fill ? v : s[i];
}

struct BwLayout {
  Layout lo;             // leave-one-out workspace (at offset 0)
  size_t o_xbar = 0, o_vecs = 0, o_lo = 0, o_fac = 0, o_coef = 0, o_rank = 0, total = 0;
  size_t rank_bytes = 0;
  int terms = 0;
};

BwLayout make_bw_layout(const tvc_tensor* A, int sweeps) {
  BwLayout b;
  b.lo = make_layout(A);
  const size_t ns = (size_t)b.lo.nsum;
  b.terms = sweeps * A->order;
  size_t o = b.lo.total;
  auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
  b.o_xbar = take(ns * 8);
  b.o_vecs = take(ns * 8);
  b.o_lo = take(ns * 8);
  b.o_fac = take((size_t)b.terms * ns * 8);
  b.o_coef = take((size_t)b.terms * 8);
  b.rank_bytes = tvc_rank_update_workspace_bytes(A->order, A->dims, b.terms);
  b.o_rank = take(b.rank_bytes);
  b.total = o;
  return b;
}

template <typename Acc>
tvc_status backward(const tvc_tensor* A, const double* xs, const double* norms, int K,
                    const double* gx, double glam, double gA_scale, void* dA, double* dx0,
                    char* ws, const BwLayout& b, hipStream_t s) {
  const Layout& Lt = b.lo;
  const int d = Lt.d;
  const i64 ns = Lt.nsum;
  double* xbar = (double*)(ws + b.o_xbar);
  double* vecs = (double*)(ws + b.o_vecs);
  double* lo = (double*)(ws + b.o_lo);
  double* fac = (double*)(ws + b.o_fac);
  double* coef = (double*)(ws + b.o_coef);
  const int g = (int)std::max<i64>(1, std::min<i64>((ns + 255) / 256, 64));
  hipLaunchKernelGGL(k_copy_f64, dim3(g), dim3(256), 0, s, gx, xbar, ns, 0.0, gx ? 0 : 1);
  const int gc = (int)std::max<int>(1, std::min<int>((b.terms + 255) / 256, 64));
  hipLaunchKernelGGL(k_copy_f64, dim3(gc), dim3(256), 0, s, (const double*)nullptr, coef,
                     (i64)b.terms, 1.0, 1);
  TVC_TRY_HIP(hipGetLastError());
  VecOffsets vo;
  vo.d = d;
  for (int m = 0; m < d; ++m) {
    vo.n[m] = Lt.n[m];
    vo.off[m] = Lt.off[m];
    vo.woff[m] = Lt.woff[m];
  }
  hopm_stats* st = (hopm_stats*)(ws + Lt.o_stats);
  Ctx c{&Lt, A, vecs, ws, st, s, nullptr};
  const uint32_t all = (d >= 32) ? 0xffffffffu : ((1u << d) - 1u);
  for (int i = K - 1; i >= 0; --i) {
    for (int j = d - 1; j >= 0; --j) {
      const int step = i * d + j;
      const double seed = (i == K - 1 && j == d - 1) ? glam : 0.0;
      hipLaunchKernelGGL(k_step_adjoint, dim3(1), dim3(kNormBlock), 0, s, xs + (size_t)i * ns,
                         xs + (size_t)(i + 1) * ns, vo, j, norms + step, seed, xbar, vecs,
                         fac + (size_t)step * ns);
      TVC_TRY_HIP(hipGetLastError());
      TVC_TRY(leave_one_out<Acc>(c, all & ~(1u << j), lo));
      hipLaunchKernelGGL(k_accumulate, dim3(g), dim3(256), 0, s, xbar, (const double*)lo, vo, j);
      TVC_TRY_HIP(hipGetLastError());
    }
  }
  if (dx0) {
    hipLaunchKernelGGL(k_copy_f64, dim3(g), dim3(256), 0, s, (const double*)xbar, dx0, ns, 0.0, 0);
    TVC_TRY_HIP(hipGetLastError());
  }
  if (dA) {
    const void* Ad = (gA_scale != 0.0) ? A->data : nullptr;
    const int32_t rs = tvc_rank_update(d, A->dims, Lt.acc_dt, Ad, gA_scale, b.terms, fac, coef,
                                       dA, ws + b.o_rank, b.rank_bytes, s);
    if (rs != TVC_OK) return (tvc_status)rs;
  }
  return TVC_OK;
}

}  // namespace
}  // namespace tvc

using namespace tvc;

extern "C" {

size_t hopm_workspace_bytes(const tvc_tensor* A) {
  if (check_tensor(A, "A") != TVC_OK || A->order < 2) return 0;
  Layout Lt = make_layout(A);
  if (A->dtype != TVC_F64 && A->dtype != TVC_F32) {
    // the same workspace must also serve the float32 refinement tensor
    tvc_tensor B = *A;
    B.dtype = TVC_F32;
    B.slab_scale = nullptr;
    Layout Lb = make_layout(&B);
    return std::max(Lt.total, Lb.total);
  }
  return Lt.total;
}

int32_t hopm_iterate(const tvc_tensor* A, double* x, int32_t sweeps, void* ws, size_t ws_bytes,
                     hopm_stats* d_stats, void* stream) {
  return iterate_any(A, x, sweeps, ws, ws_bytes, d_stats, (hipStream_t)stream);
}

int32_t hopm_solve(const tvc_tensor* A, const tvc_tensor* A_refine, double* x, double tol,
                   int32_t max_sweeps, int32_t check_every, int32_t refine_sweeps, void* ws,
                   size_t ws_bytes, hopm_stats* h_out, void* stream) {
  TVC_TRY(check_tensor(A, "A"));
  if (A->order < 2) return fail(TVC_EINVAL, "HOPM needs order >= 2");
  if (!h_out) return fail(TVC_EINVAL, "h_out is NULL");
  if (max_sweeps < 1 || check_every < 1) return fail(TVC_EINVAL, "max_sweeps and check_every must be >= 1");
  if (!(tol >= 0.0)) return fail(TVC_EINVAL, "tol must be >= 0");
  if (A_refine) {
    TVC_TRY(check_tensor(A_refine, "A_refine"));
    if (A_refine->dtype != TVC_F32) return fail(TVC_EDTYPE, "A_refine must be TVC_F32");
    if (A_refine->order != A->order) return fail(TVC_EINVAL, "A_refine dims differ from A");
    for (int i = 0; i < A->order; ++i)
      if (A_refine->dims[i] != A->dims[i]) return fail(TVC_EINVAL, "A_refine dims differ from A");
    if (refine_sweeps < 0) return fail(TVC_EINVAL, "refine_sweeps must be >= 0");
  }
  Layout Lt = make_layout(A);
  if (ws_bytes < hopm_workspace_bytes(A))
    return fail(TVC_EWORKSPACE, "HOPM workspace too small");
  // device stats live in the first slot of the workspace
  hopm_stats* dst = (hopm_stats*)((char*)ws + Lt.o_stats);
  hipStream_t s = (hipStream_t)stream;
  hopm_stats h{};
  // The per-check read-back goes straight into h_out when the caller's
  // record is pinned host memory (a copy to pageable memory is staged and
  // costs tens of microseconds per check), else into a local record.
  hopm_stats* rb = &h;
  {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, h_out) == hipSuccess && at.type == hipMemoryTypeHost) rb = h_out;
    (void)hipGetLastError();  // an unregistered pointer reports an error: not ours to keep
  }
  bool converged = false;
  int done = 0;
  while (done < max_sweeps) {
    const int k = std::min(check_every, max_sweeps - done);
    TVC_TRY(iterate_any(A, x, k, ws, ws_bytes, dst, s));
    TVC_TRY_HIP(hipMemcpyAsync(rb, dst, sizeof(h), hipMemcpyDeviceToHost, s));
    TVC_TRY_HIP(hipStreamSynchronize(s));
    h = *rb;
    done += k;
    if (h.status != TVC_OK) {
      h.sweeps = done;
      *h_out = h;
      return fail(TVC_EDEGENERATE, "zero-norm vector during HOPM");
    }
    if (h.delta < tol) {
      converged = true;
      break;
    }
  }
  h.sweeps = done;
  int rdone = 0;
  if (A_refine && refine_sweeps > 0) {
    // the refinement is the last stage: its own stopping test decides the
    // status, whether or not the low-precision stage met tol
    converged = false;
    hopm_stats hr{};
    while (rdone < refine_sweeps) {
      const int k = std::min(check_every, refine_sweeps - rdone);
      TVC_TRY(iterate_any(A_refine, x, k, ws, ws_bytes, dst, s));
      TVC_TRY_HIP(hipMemcpyAsync(rb, dst, sizeof(hr), hipMemcpyDeviceToHost, s));
      TVC_TRY_HIP(hipStreamSynchronize(s));
      hr = *rb;
      rdone += k;
      if (hr.status != TVC_OK) {
        h.status = hr.status;
        h.refine_sweeps = rdone;
        *h_out = h;
        return fail(TVC_EDEGENERATE, "zero-norm vector during refinement");
      }
      h.lambda = hr.lambda;
      h.delta = hr.delta;
      if (hr.delta < tol) {
        converged = true;
        break;
      }
    }
  }
  h.refine_sweeps = rdone;
  *h_out = h;
  if (!converged)
    return fail(TVC_ENOTCONVERGED, rdone ? "refine_sweeps reached before delta < tol"
                                          : "max_sweeps reached before delta < tol");
  return TVC_OK;
}

int32_t hopm_jacobi_iterate(const tvc_tensor* A, double* x, int32_t sweeps, void* ws,
                            size_t ws_bytes, hopm_stats* d_stats, void* stream) {
  return iterate_any(A, x, sweeps, ws, ws_bytes, d_stats, (hipStream_t)stream, nullptr, true);
}

int32_t hopm_jacobi_solve(const tvc_tensor* A, double* x, double tol, int32_t max_sweeps,
                          int32_t check_every, void* ws, size_t ws_bytes, hopm_stats* h_out,
                          void* stream) {
  TVC_TRY(check_tensor(A, "A"));
  if (A->order < 2) return fail(TVC_EINVAL, "HOPM needs order >= 2");
  if (!h_out) return fail(TVC_EINVAL, "h_out is NULL");
  if (max_sweeps < 1 || check_every < 1) return fail(TVC_EINVAL, "max_sweeps and check_every must be >= 1");
  if (!(tol >= 0.0)) return fail(TVC_EINVAL, "tol must be >= 0");
  Layout Lt = make_layout(A);
  if (ws_bytes < Lt.total) return fail(TVC_EWORKSPACE, "HOPM workspace too small");
  hopm_stats* dst = (hopm_stats*)((char*)ws + Lt.o_stats);
  hipStream_t s = (hipStream_t)stream;
  hopm_stats h{};
  hopm_stats* rb = &h;
  {
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, h_out) == hipSuccess && at.type == hipMemoryTypeHost) rb = h_out;
    (void)hipGetLastError();
  }
  int done = 0;
  while (done < max_sweeps) {
    const int k = std::min(check_every, max_sweeps - done);
    TVC_TRY(iterate_any(A, x, k, ws, ws_bytes, dst, s, nullptr, true));
    TVC_TRY_HIP(hipMemcpyAsync(rb, dst, sizeof(h), hipMemcpyDeviceToHost, s));
    TVC_TRY_HIP(hipStreamSynchronize(s));
    h = *rb;
    done += k;
    h.sweeps = done;
    h.refine_sweeps = 0;
    if (h.status != TVC_OK) {
      *h_out = h;
      return fail(TVC_EDEGENERATE, "zero-norm vector during HOPM");
    }
    if (h.delta < tol) {
      *h_out = h;
      return TVC_OK;
    }
  }
  *h_out = h;
  return fail(TVC_ENOTCONVERGED, "max_sweeps reached before delta < tol");
}

int32_t hopm_iterate_record(const tvc_tensor* A, double* x, int32_t sweeps, void* ws,
                            size_t ws_bytes, hopm_stats* d_stats, double* d_norms, void* stream) {
  if (!d_norms) return fail(TVC_EINVAL, "d_norms is NULL");
  return iterate_any(A, x, sweeps, ws, ws_bytes, d_stats, (hipStream_t)stream, d_norms);
}

int32_t tvc_leave_one_out(const tvc_tensor* A, const double* v, uint32_t modes, double* out,
                          void* ws, size_t ws_bytes, void* stream) {
  TVC_TRY(check_tensor(A, "A"));
  if (A->order < 2) return fail(TVC_EINVAL, "leave-one-out needs order >= 2");
  if (!v || !out) return fail(TVC_EINVAL, "v or out is NULL");
  if ((uintptr_t)v % 8 || (uintptr_t)out % 8) return fail(TVC_EINVAL, "v or out misaligned");
  Layout Lt = make_layout(A);
  TVC_TRY(check_hopm_args(A, const_cast<double*>(v), ws, ws_bytes, Lt));
  const size_t vb = (size_t)Lt.nsum * 8;
  if (overlaps(out, vb, v, vb) || overlaps(out, vb, ws, ws_bytes) ||
      overlaps(out, vb, A->data, (size_t)numel(A) * elem_bytes(A->dtype)))
    return fail(TVC_EALIAS, "out overlaps v, the workspace or A");
  const uint32_t all = A->order >= 32 ? 0xffffffffu : ((1u << A->order) - 1u);
  if (modes & ~all) return fail(TVC_EINVAL, "modes has bits beyond the order");
  hopm_stats* st = (hopm_stats*)((char*)ws + Lt.o_stats);
  Ctx c{&Lt, A, const_cast<double*>(v), (char*)ws, st, (hipStream_t)stream, nullptr};
  if (A->dtype == TVC_F64) return leave_one_out<double>(c, modes, out);
  return leave_one_out<float>(c, modes, out);
}

size_t hopm_backward_workspace_bytes(const tvc_tensor* A, int32_t sweeps) {
  if (check_tensor(A, "A") != TVC_OK || A->order < 2 || sweeps < 1) return 0;
  return make_bw_layout(A, sweeps).total;
}

int32_t hopm_backward(const tvc_tensor* A, const double* xs, const double* norms, int32_t sweeps,
                      const double* gx, double glam, double gA_scale, void* dA, double* dx0,
                      void* ws, size_t ws_bytes, void* stream) {
  TVC_TRY(check_tensor(A, "A"));
  if (A->order < 2) return fail(TVC_EINVAL, "HOPM needs order >= 2");
  if (sweeps < 1) return fail(TVC_EINVAL, "sweeps must be >= 1");
  if (!xs || !norms) return fail(TVC_EINVAL, "xs or norms is NULL");
  if (!dA && !dx0) return fail(TVC_EINVAL, "nothing to compute (dA and dx0 are NULL)");
  if (gA_scale != 0.0 && A->dtype != TVC_F32 && A->dtype != TVC_F64)
    return fail(TVC_EDTYPE, "gA_scale != 0 needs a TVC_F32 or TVC_F64 tensor");
  BwLayout b = make_bw_layout(A, sweeps);
  if (!ws || ws_bytes < b.total || (uintptr_t)ws % 256)
    return fail(TVC_EWORKSPACE, "workspace of " + std::to_string(b.total) + " bytes required");
  const size_t abytes = (size_t)numel(A) * elem_bytes(A->dtype);
  const size_t dbytes = (size_t)numel(A) * acc_bytes(A->dtype);
  if (overlaps(ws, ws_bytes, A->data, abytes) || (dA && overlaps(dA, dbytes, ws, ws_bytes)))
    return fail(TVC_EALIAS, "workspace overlaps A or dA");
  if (dA && dA != A->data && overlaps(dA, dbytes, A->data, abytes))
    return fail(TVC_EALIAS, "dA overlaps A");
  if (A->dtype == TVC_F64)
    return backward<double>(A, xs, norms, sweeps, gx, glam, gA_scale, dA, dx0, (char*)ws, b,
                            (hipStream_t)stream);
  return backward<float>(A, xs, norms, sweeps, gx, glam, gA_scale, dA, dx0, (char*)ws, b,
                         (hipStream_t)stream);
}

}  // extern "C"
