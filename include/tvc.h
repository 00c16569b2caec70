/*
 * tvc.h -- C ABI of the MI355X (gfx950) tensor-vector contraction library.
 *
 * Operations (Martinez-Ferrer, Yzelman, Beltran, "Distributed and
 * heterogeneous tensor-vector contraction algorithms for high performance
 * computing", FGCS 2025, arXiv 2501.03121):
 *   - the k-mode tensor-vector contraction Y = A x_k x of a dense order-d
 *     tensor (Sec. 3), with the BLAS-like alpha/beta scaling of Eq. (1);
 *   - the higher-order power method (HOPM, Sec. 3) with the Gauss-Seidel
 *     update order of Algorithm 1 (dHOPM_3), on one device;
 *   - storage of A in a lower precision with promotion before arithmetic
 *     (Sec. 5.5), plus derivatives and batched HOPM built on the same kernels.
 *
 * Conventions shared by every entry point
 *   Layout     Tensors are dense, C-contiguous and last-order (the last mode
 *              varies fastest), zero-based, as in Sec. 3.  The contraction
 *              output keeps the remaining modes in their original order.
 *   Memory     Every data pointer is a DEVICE pointer owned by the caller,
 *              unless stated as host.  The library never allocates device
 *              memory; scratch space is passed in as a workspace whose size
 *              the matching *_workspace_bytes call returns.
 *   Streams    `stream` is a hipStream_t passed as void* (NULL = the null
 *              stream).  All work is enqueued asynchronously on it; only
 *              hopm_solve waits on the stream.
 *   Dtypes     A: TVC_F64, TVC_F32, TVC_F16 (IEEE binary16), TVC_BF16,
 *              TVC_F8E4M3 (OCP E4M3FN, with one float32 scale per mode-0
 *              slice).  Vectors x, outputs y and gradients are double for
 *              TVC_F64 and float for every other dtype.  Accumulation is in
 *              double for TVC_F64 and float otherwise.  HOPM vectors are
 *              always double.
 *   Errors     Every call returns a tvc_status; nothing aborts or throws.
 *              On error nothing is enqueued.  tvc_last_error() gives a
 *              message for the last failure of the calling thread.
 */
#ifndef TVC_H
#define TVC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TVC_OK = 0,
  TVC_EINVAL = 1,        /* bad order, dims, mode, size or pointer */
  TVC_EDTYPE = 2,        /* dtype not valid for this entry point */
  TVC_EALIAS = 3,        /* an output overlaps an input */
  TVC_EWORKSPACE = 4,    /* workspace NULL, misaligned or too small */
  TVC_EHIP = 5,          /* a HIP runtime call or kernel launch failed */
  TVC_EDEGENERATE = 6,   /* a vector to normalise had zero norm */
  TVC_ENOTCONVERGED = 7  /* a sweep cap reached before delta < tol */
} tvc_status;

typedef enum {
  TVC_F64 = 0,
  TVC_F32 = 1,
  TVC_F16 = 2,
  TVC_BF16 = 3,
  TVC_F8E4M3 = 4
} tvc_dtype;

#define TVC_MAX_ORDER 16

/* A dense tensor.  order in [1, TVC_MAX_ORDER]; dims[0..order) >= 1; the
 * element count must fit in int64.  data must be aligned to the element size
 * (16-byte alignment enables the vector-load kernels).  slab_scale: for
 * TVC_F8E4M3, dims[0] float32 scales, the value of element (i0, ...) being
 * decode(code) * slab_scale[i0]; NULL for every other dtype. */
typedef struct {
  int32_t order;
  int32_t dtype;                 /* tvc_dtype */
  int64_t dims[TVC_MAX_ORDER];
  const void* data;
  const float* slab_scale;
} tvc_tensor;

/* HOPM progress record (device-resident for hopm_iterate, host for
 * hopm_solve).  lambda = norm of the last contraction result before its
 * normalisation (= A x_0 x_0 ... x_{d-1} x_{d-1} afterwards); delta = largest
 * ||x_j(new) - x_j(old)||_2 over j in the last sweep; sweeps = sweeps done by
 * the call; status = TVC_OK or TVC_EDEGENERATE; refine_sweeps = sweeps of the
 * refinement stage of hopm_solve (0 otherwise). */
typedef struct {
  double lambda;
  double delta;
  int32_t sweeps;
  int32_t status;
  int32_t refine_sweeps;
  int32_t reserved;
} hopm_stats;

/* Human-readable name of a status code (static string). */
const char* tvc_status_string(int32_t status);

/* Detail message of the last failing call on this thread ("" if none). */
const char* tvc_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t tvc_version(void);

/* ---------------------------------------------------------------------------
 * Tensor-vector contraction, Sec. 3 (definition and the (u, n_k, v) view)
 * and Eq. (1) (alpha/beta form):
 *     Y := alpha * (A x_mode x) + beta * Y
 * x: n_mode elements.  y: N / n_mode elements, C-contiguous over the modes of
 * A without `mode`.  beta == 0 means y is not read (NaN in y is harmless).
 * ws/ws_bytes: scratch of at least tvc_contract_workspace_bytes(A, mode)
 * bytes, 256-byte aligned; may be NULL when that size is 0.
 * Errors: EINVAL (order/dims/mode/pointers), EDTYPE (unknown dtype, or
 * TVC_F8E4M3 without slab_scale), EALIAS (y overlaps A or x), EWORKSPACE,
 * EHIP.  Results are deterministic: the same call gives the same bits.
 * ------------------------------------------------------------------------- */
size_t tvc_contract_workspace_bytes(const tvc_tensor* A, int32_t mode);
int32_t tvc_contract(const tvc_tensor* A, int32_t mode, const void* x, void* y,
                     double alpha, double beta, void* ws, size_t ws_bytes,
                     void* stream);

/* tvc_contract without a workspace argument, for callers that cannot
 * allocate device memory (code under hipGraph capture, serving loops that
 * forbid allocation): the scratch lives in a fixed device array of
 * tvc_contract_noalloc_max_scratch() bytes (8 MiB) that the library holds on
 * each device it runs on, until the process ends.  Makes no allocation.
 * Same arguments, results and errors as tvc_contract, plus EWORKSPACE when
 * tvc_contract_workspace_bytes(A, mode) exceeds that size (the contraction
 * is not run).  Every call on one device shares that device's array: calls
 * that overlap in time on one device (two streams, two threads) race and
 * must not be made; calls in order on one stream are safe. */
size_t tvc_contract_noalloc_max_scratch(void);
int32_t tvc_contract_noalloc(const tvc_tensor* A, int32_t mode, const void* x, void* y,
                             double alpha, double beta, void* stream);

/* Introspection of the launch tvc_contract(A, mode, ...) would make, for
 * tests, benchmarks and the autotuner.  Writes up to n values to info (host):
 * [0] family (0 = rows of the right-extent-1 view, 1 = column streaming,
 * 2 = small-right slabs, 3 = small slabs staged through LDS), [1] 1 if
 * 16-byte vector loads are used, [2] wave
 * groups per workgroup along the contracted extent (family 1), [3] number
 * of splits of the contracted extent (> 1 adds a finalize kernel), [4]
 * workgroups launched, [5] lanes per row (families 0 and 2, 0 = a wave per
 * row; family 3: lanes per output), [6] elements of each contiguous row after its last whole 16-byte
 * vector (vector path only; such rows need only start on a 4-byte
 * boundary), [7] full 16-byte vectors (or elements, scalar path) per row,
 * [8] 1 if each workgroup collects its outputs in an LDS window and writes
 * them in bursts (short contracted extents, where y is a sizeable share of
 * the traffic), [9] family 1: column units per lane of the column-strip
 * kernel (a wave per strip of 64 times that many units), 0 for wave groups
 * sharing column tiles, [10] 1 if the column-strip kernel's workgroups
 * start their rows at different row indices (rows 1-64 MB apart), [11]
 * family 3: slabs per block copied through the 32 KB LDS staging buffer
 * (the block and the M weights share it), 0 otherwise.
 * Returns TVC_OK or an argument error. */
int32_t tvc_contract_plan(const tvc_tensor* A, int32_t mode, int32_t* info, int32_t n);

/* ---------------------------------------------------------------------------
 * Higher-order power method, Sec. 3 (canonical HOPM) with the update order
 * of Algorithm 1: external iteration j = 0..d-1 replaces x_j by the
 * normalised contraction of A with every other vector, using the vectors
 * already updated in the same sweep.  One sweep streams A twice: once to
 * form M = A contracted over modes 2..d-1 (which gives x_0 and x_1), once to
 * form A contracted over modes 0 and 1 (which gives x_2..x_{d-1}).  Needs
 * order >= 2.
 * x: device double buffer holding x_0, x_1, ..., x_{d-1} back to back
 * (sum of dims elements), unit-norm on entry, updated in place.
 * ws: at least hopm_workspace_bytes(A) bytes, 256-byte aligned.  The same
 * workspace size also serves a TVC_F32 tensor of the same dims.
 * ------------------------------------------------------------------------- */
size_t hopm_workspace_bytes(const tvc_tensor* A);

/* Runs exactly `sweeps` (>= 1) sweeps; no host synchronisation, safe to
 * capture in a hipGraph.  d_stats (device) receives lambda and delta of the
 * last sweep, sweeps = `sweeps`, status TVC_EDEGENERATE if any zero-norm
 * vector was met (that vector is then left unchanged). */
int32_t hopm_iterate(const tvc_tensor* A, double* x, int32_t sweeps, void* ws,
                     size_t ws_bytes, hopm_stats* d_stats, void* stream);

/* Sweeps on A until delta < tol (tested every `check_every` sweeps, which
 * reads the stats back to the host and synchronises the stream) or
 * max_sweeps sweeps.  Then, if A_refine is not NULL (a TVC_F32 tensor of the
 * same dims, normally the original of a low-precision A) and refine_sweeps
 * > 0, a refinement stage: up to refine_sweeps sweeps on A_refine with the
 * same stopping test, whether or not the first stage met tol.  h_out (host)
 * receives the final record: sweeps of the first stage, refine_sweeps of the
 * refinement, lambda and delta of the last sweep run.  When h_out is pinned
 * host memory (hipHostMalloc), each check reads the record back straight
 * into it, which is faster than the staged copy pageable memory needs.
 * Returns TVC_OK when the last stage that ran (the refinement if there is
 * one) ended with delta < tol; TVC_ENOTCONVERGED when it stopped at its
 * sweep cap instead (the last iterate is still in x); TVC_EDEGENERATE; or an
 * argument error. */
int32_t hopm_solve(const tvc_tensor* A, const tvc_tensor* A_refine, double* x,
                   double tol, int32_t max_sweeps, int32_t check_every,
                   int32_t refine_sweeps, void* ws, size_t ws_bytes,
                   hopm_stats* h_out, void* stream);

/* Jacobi HOPM, a variant of the method (not the paper's sweep, which is
 * Gauss-Seidel): in every sweep each x_j is replaced by the normalised
 * contraction of A with the OTHER vectors of the previous sweep, so all d
 * contractions come from one pass over A (half the bytes of a Gauss-Seidel
 * sweep; usually more sweeps to converge).  Each new x_j takes the sign that
 * keeps <x_j(new), x_j(old)> >= 0 (the directions are those of the plain
 * Jacobi iteration; without the choice, even orders can flip every sign in
 * every sweep and delta would not fall).  Same arguments, workspace
 * (hopm_workspace_bytes), stats and errors as hopm_iterate / hopm_solve
 * (no refinement stage); lambda = norm of the contraction for x_{d-1}.
 * No host synchronisation in hopm_jacobi_iterate. */
int32_t hopm_jacobi_iterate(const tvc_tensor* A, double* x, int32_t sweeps, void* ws,
                            size_t ws_bytes, hopm_stats* d_stats, void* stream);
int32_t hopm_jacobi_solve(const tvc_tensor* A, double* x, double tol, int32_t max_sweeps,
                          int32_t check_every, void* ws, size_t ws_bytes, hopm_stats* h_out,
                          void* stream);

/* ---------------------------------------------------------------------------
 * Lower-precision storage (Sec. 5.5: values stored narrow, promoted before
 * arithmetic).  Converts a TVC_F32 tensor `src` into `dst_dtype` (TVC_F16,
 * TVC_BF16 or TVC_F8E4M3), written to dst (N elements of the narrow type).
 * Rounding is to nearest even; flags & TVC_QUANT_TRUNCATE selects bf16 by
 * truncation instead (the paper's conversion).  For TVC_F8E4M3 the
 * per-mode-0-slice scale absmax/448 (1 for an all-zero slice) is written to
 * slab_scale_out (dims[0] floats) and codes are e4m3(src / scale), finite
 * overflow saturating to +-448.  Errors: EINVAL, EDTYPE, EALIAS, EHIP.
 * ------------------------------------------------------------------------- */
#define TVC_QUANT_TRUNCATE 1
int32_t tvc_quantize(const tvc_tensor* src, void* dst, int32_t dst_dtype,
                     float* slab_scale_out, int32_t flags, void* stream);

/* ---------------------------------------------------------------------------
 * Derivatives of Y = A x_k x (Sec. 3 definition) for an incoming gradient g
 * of Y (N / n_k elements in the layout of y):
 *   dx[m] = sum of A[.., m, ..] * g[..] over every other index
 *           (A contracted with g over every mode except k), n_k elements;
 *   dA    = alpha * (g outer x placed at mode k) + beta * dA, N elements
 *           (beta == 0: dA is not read).
 * tvc_backward_x: A of any dtype; g and dx are double for TVC_F64, float
 * otherwise; one pass over A.  ws: tvc_backward_x_workspace_bytes(A, mode)
 * bytes, 256-byte aligned (NULL when 0).
 * tvc_backward_A: `dtype` (TVC_F32 or TVC_F64) is the type of g, x and dA.
 * Errors: EINVAL, EDTYPE, EALIAS, EWORKSPACE, EHIP.
 * ------------------------------------------------------------------------- */
size_t tvc_backward_x_workspace_bytes(const tvc_tensor* A, int32_t mode);
int32_t tvc_backward_x(const tvc_tensor* A, int32_t mode, const void* g, void* dx,
                       void* ws, size_t ws_bytes, void* stream);
int32_t tvc_backward_A(int32_t order, const int64_t* dims, int32_t dtype,
                       int32_t mode, const void* g, const void* x, void* dA,
                       double alpha, double beta, void* stream);

/* Leave-one-out contractions (the operands of the HOPM update of Sec. 3, and
 * of its derivative): with vectors v_0..v_{d-1} (device double, back to back
 * as in hopm_iterate) it writes, for every mode m in the bit set `modes`,
 *   out_m = A contracted with v_k over every k != m
 * into out (device double, back to back; entries of other modes untouched).
 * At most two passes over A.  ws: hopm_workspace_bytes(A) bytes. */
int32_t tvc_leave_one_out(const tvc_tensor* A, const double* v, uint32_t modes,
                          double* out, void* ws, size_t ws_bytes, void* stream);

/* Dense rank-R update: D := alpha * A + sum_r c_r f_{r,0} o ... o f_{r,d-1}
 * over tensors of dims `dims` whose elements are `dtype` (TVC_F32 or
 * TVC_F64); A may equal D, and may be NULL when alpha == 0.  factors: device
 * double, R blocks of sum(dims) values (the factor vectors of term r back to
 * back); coef: device double, R values.  R <= 4096.
 * ws: tvc_rank_update_workspace_bytes(order, dims, R) bytes. */
size_t tvc_rank_update_workspace_bytes(int32_t order, const int64_t* dims, int32_t R);
int32_t tvc_rank_update(int32_t order, const int64_t* dims, int32_t dtype, const void* A,
                        double alpha, int32_t R, const double* factors,
                        const double* coef, void* D, void* ws, size_t ws_bytes,
                        void* stream);

/* hopm_iterate that also stores the pre-normalisation norm ||y|| of every
 * (sweep, j) step: d_norms (device double) receives sweeps * order values,
 * step (i, j) at i * order + j. */
int32_t hopm_iterate_record(const tvc_tensor* A, double* x, int32_t sweeps, void* ws,
                            size_t ws_bytes, hopm_stats* d_stats, double* d_norms,
                            void* stream);

/* Reverse pass through K HOPM sweeps (the derivative of unrolled HOPM).
 * xs: device double, (K + 1) blocks of sum(dims) values: the vectors before
 * sweep 0 and after every sweep (the checkpoints; the state before any step
 * (i, j) is rebuilt from blocks i and i + 1).  norms: the K * order values
 * of hopm_iterate_record.  gx: adjoint of the final vectors (sum(dims)
 * doubles, or NULL for zero); glam: adjoint of the final lambda.
 * Outputs (either may be NULL, not both): dA (N values, double for TVC_F64,
 * float otherwise) := gA_scale * A + the gradient with respect to A, formed
 * as K * order rank-1 terms and written once; dx0 (double, sum(dims)): the
 * gradient with respect to the initial vectors.  Each step costs one
 * leave-one-out call (two passes over A).  gA_scale != 0 needs a TVC_F32 or
 * TVC_F64 tensor.  ws: hopm_backward_workspace_bytes(A, K) bytes. */
size_t hopm_backward_workspace_bytes(const tvc_tensor* A, int32_t sweeps);
int32_t hopm_backward(const tvc_tensor* A, const double* xs, const double* norms,
                      int32_t sweeps, const double* gx, double glam, double gA_scale,
                      void* dA, double* dx0, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Batched HOPM (Sec. 3 HOPM, update order of Algorithm 1): many independent
 * TVC_F32 instances of order 3..8 and uneven shapes, all swept `sweeps`
 * times by one persistent kernel launch.  Each sweep of an instance is
 * split into tiled passes over its tensor and single-workgroup vector
 * steps; work items are (instance, phase, tile, sweep) in a device queue,
 * and each instance advances through its phases on its own.  No host
 * synchronisation: safe to capture in a hipGraph.
 *
 * The caller fills, per instance, A (device, dense last-order float32), x
 * (device, double, the unit vectors back to back, updated in place), dims,
 * order, and optionally tile_rows1 / tile_rows2 (rows of the [n0 n1][rest]
 * view per work item of the two passes; 0 = derived from tile_elems).
 * hopm_batch_prepare (host) completes the records (nt1, nt2, ws_offset,
 * init_slot) and the plan; instances start in the given order (put the
 * largest first).  The caller then copies the records to device memory and
 * calls hopm_batch_run with a workspace of plan->ws_bytes bytes (256-byte
 * aligned) and `count` device hopm_stats records.  grid = 0 picks 4
 * workgroups per compute unit.  Every wait inside the kernel is bounded;
 * hopm_batch_error copies the workspace's error word (0 = none) to a device
 * uint32 after a run.  Calls sharing a workspace must not overlap.
 * ------------------------------------------------------------------------- */
typedef struct {
  const float* A;
  double* x;
  int64_t dims[8];
  int32_t order;
  int32_t tile_rows1;
  int32_t tile_rows2;
  int32_t nt1;             /* filled by hopm_batch_prepare */
  int32_t nt2;             /* filled by hopm_batch_prepare */
  int32_t reserved;
  int64_t ws_offset;       /* filled by hopm_batch_prepare */
  int64_t init_slot;       /* filled by hopm_batch_prepare */
} hopm_batch_desc;

typedef struct {
  int64_t queue_slots;
  int64_t initial_items;
  size_t ws_bytes;
  int32_t count;
  int32_t sweeps;
} hopm_batch_plan;

int32_t hopm_batch_prepare(hopm_batch_desc* descs, int32_t count, int32_t sweeps,
                           int32_t tile_elems, hopm_batch_plan* plan);
int32_t hopm_batch_run(const hopm_batch_desc* d_descs, const hopm_batch_plan* plan,
                       int32_t grid, void* ws, size_t ws_bytes, hopm_stats* d_stats,
                       void* stream);
int32_t hopm_batch_error(const void* ws, uint32_t* d_error_out, void* stream);

/* Profile of the last hopm_batch_run on this workspace: copies six uint64
 * values to device memory d_out (asynchronously on `stream`): work items
 * run; wall-clock ticks (100 MHz) summed over workgroups spent claiming a
 * queue slot and waiting for it to be published; and ticks spent running
 * items of each of the four phases (pass-1 tiles, the x_0/x_1 step, pass-2
 * tiles, the W chain).  The waiting share shows how much of the persistent
 * grid idles on the dependencies between phases.  Returns TVC_OK,
 * TVC_EINVAL for NULL pointers or TVC_EHIP. */
int32_t hopm_batch_profile(const void* ws, uint64_t* d_out, void* stream);

/* ---------------------------------------------------------------------------
 * Tuning (used by the autotuner): override launch parameters the dispatcher
 * picks for one kernel family: 0 = rows (right extent 1), 1 = column
 * streaming, 2 = small-right slabs, 3 = small slabs staged through LDS.
 * blocks_per_cu caps the persistent grid at that many 256-thread workgroups
 * per compute unit; for family 3 a negative value turns the family off (the
 * dispatcher then uses families 0 and 2 for those shapes).  split_m (family
 * 1 only: 1, 2 or 4) is the number of wave groups sharing one column tile;
 * a negative split_m selects the plain kernels: no LDS output window in any
 * family (outputs are stored as each task finishes) and no column strips
 * (family 1 always uses wave groups sharing column tiles).  Values of 0
 * restore the built-in choice.  family 4 selects how the first pass of a
 * HOPM sweep contracts its rows: blocks_per_cu > 0 always as strips of
 * columns whose weights stay in registers, < 0 never, 0 the built-in
 * rule.  Process-wide; set it while no
 * other thread is launching contractions.
 * ------------------------------------------------------------------------- */
int32_t tvc_set_tuning(int32_t family, int32_t blocks_per_cu, int32_t split_m);

/* ---------------------------------------------------------------------------
 * Bandwidth probes (the analogue of the paper's STREAM yardstick, Sec. 5.1,
 * written for this library): read `bytes` bytes of src and write one float
 * per workgroup to sink (>= grid floats), or copy `bytes` bytes from src to
 * dst.  bytes must be a multiple of 16; pointers 16-byte aligned.  grid = 0
 * picks a default.
 * ------------------------------------------------------------------------- */
int32_t tvc_probe_read(const void* src, size_t bytes, float* sink, int32_t grid,
                       void* stream);
int32_t tvc_probe_copy(const void* src, void* dst, size_t bytes, int32_t grid,
                       void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TVC_H */
