#!/usr/bin/env python3
"""Benchmark of the TVC / HOPM hot path on one MI355X.

One step = the k-mode contraction of a 1024^3 and a 32^6 float32 tensor
(N(0,1) entries) in every mode (3 + 6 contractions), plus one HOPM sweep on
each of two planted tensors of the same shapes (10 * a o b o c ... + N(0, 0.1^2)).
`value` is the algorithmic HBM traffic of the whole step divided by its time:
a contraction moves N*4 bytes of A plus its vector and output; a sweep moves
2*N*4 bytes (two passes over A) plus the vectors.  Inputs are resident in HBM
before timing starts.

Printed: one JSON line (the last line of stdout).  Extra fields report the
per-mode figures, the narrow storage formats, float64 at the same shapes,
time to solution (float32, bf16, fp16, E4M3, bf16 with float32 refinement,
Jacobi sweeps) with every result's error against the float64 oracle, the
looped rocBLAS comparator, the bandwidth probe, derivatives, the batch, the
paper's Table 1 tensors, the dominant kernel against the HBM roofline and
the float64 CPU oracle.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "TVC & HOPM-sweep HBM GB/s (% of peak), bf16 vs fp32 at stated rel err"
SHAPES = [(1024, 1024, 1024), (32, 32, 32, 32, 32, 32)]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def tvc_bytes(dims, k, b_a, b_v=4):
    n = math.prod(dims)
    return n * b_a + (n // dims[k]) * b_v + dims[k] * b_v


def sweep_bytes(dims, b_a):
    return 2 * math.prod(dims) * b_a + 8 * sum(dims)


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, or None if the kernel source has
    changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "tvc_colw_f32_32p6_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, KeyError, ValueError):
        return None
    return int(rec["traffic_bytes_per_launch"]) if sha == rec["source_sha256"] else None


class Call:
    """A prepared C-ABI call (descriptors built once, outside the timed loop)."""

    def __init__(self, fn, *args):
        self.fn = fn
        self.args = args

    def __call__(self):
        st = self.fn(*self.args)
        if st != 0:
            from paper_2501_03121_amd import _lib
            _lib.check(st)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--calib", action="store_true",
                    help="only run the read/copy probes of known size (counter calibration)")
    ap.add_argument("--no-table1", action="store_true", help="skip the Table 1 leg of the extras")
    ap.add_argument("--focus", default="",
                    help="only repeat one operation (for profilers): tvc:FMT:SHAPE:MODE, sweep:FMT:SHAPE, "
                         "jacobi:FMT:SHAPE or solve:FMT:SHAPE, with FMT in f64/f32/f16/bf16/e4m3 and SHAPE "
                         "such as 32^6 or 1024^3")
    ap.add_argument("--reps", type=int, default=20, help="repetitions of --focus")
    ap.add_argument("--tune", action="append", default=[],
                    help="FAMILY:BLOCKS_PER_CU:SPLIT_M passed to tvc_set_tuning before anything runs")
    ap.add_argument("--table1", action="store_true",
                    help="only the hypersquare tensors of the paper's Table 1 (orders 2-10, float32): "
                         "contraction in every mode and one HOPM sweep, %% of peak mean and std per order")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the contraction shards along a non-contracted mode without communication; only one device is measured here)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import _lib as L
    from paper_2501_03121_amd import core, synth

    global T0
    T0 = time.perf_counter()
    dev = torch.device("cuda:0")
    lib = L.lib()
    for t in args.tune:
        f, b, m = (int(v) for v in t.split(":"))
        L.check(lib.tvc_set_tuning(f, b, m))
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    if args.calib:
        # 1 GiB read and 1 GiB -> 1 GiB copy, twice each
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        sink = torch.empty(8192, dtype=torch.float32, device=dev)
        for _ in range(2):
            tvc.probe_read(a, sink)
            tvc.probe_copy(a, b)
        torch.cuda.synchronize()
        print(json.dumps({"calib": {"read_bytes": a.numel() * 4, "copy_read_bytes": a.numel() * 4,
                                    "copy_write_bytes": a.numel() * 4}}), flush=True)
        return 0

    if args.table1:
        print(json.dumps({"table1": run_table1(dev), "table1_f64": run_table1(dev, dtype="f64")}), flush=True)
        return 0

    if args.focus:
        print(json.dumps({"focus": run_focus(args.focus, args.reps, dev)}), flush=True)
        return 0

    # ------------------------------------------------------------ inputs
    log("generating inputs")
    T = [synth.device_normal(s, 100 + 10 * i, dev) for i, s in enumerate(SHAPES)]
    Hs, planted = [], []
    for i, s in enumerate(SHAPES):
        A, a = synth.device_planted(s, 10.0, 0.1, 200 + 10 * i, dev)
        Hs.append(A)
        planted.append(a)
    torch.cuda.synchronize()

    # contraction calls (x unit uniform vectors, outputs preallocated)
    tvc_calls = []   # (label, Call, bytes, plan)
    keep = []
    for i, (A, s) in enumerate(zip(T, SHAPES)):
        desc = core.describe(A)
        keep.append(desc)
        for k in range(len(s)):
            x = torch.from_numpy(synth.unit_vectors([s[k]], 300 + k)[0]).float().to(dev)
            y = torch.empty(A.numel() // s[k], dtype=torch.float32, device=dev)
            keep += [x, y]
            need = lib.tvc_contract_workspace_bytes(desc, k)
            ws = torch.empty(need + 256, dtype=torch.uint8, device=dev) if need else None
            keep.append(ws)
            wp = ((ws.data_ptr() + 255) & ~255) if ws is not None else None
            c = Call(lib.tvc_contract, desc, k, x.data_ptr(), y.data_ptr(), 1.0, 0.0, wp, need, sh)
            tvc_calls.append((f"{len(s)}d_{s[0]}_mode{k}", c, tvc_bytes(s, k, 4),
                              tvc.contract_plan(A, k)))

    # HOPM sweep calls (warm start, vectors float64, workspace + stats preallocated)
    hopm_calls = []
    for i, (A, s) in enumerate(zip(Hs, SHAPES)):
        desc = core.describe(A)
        keep.append(desc)
        x = tvc.pack_vectors(synth.warm_start(planted[i], 0.9, 400 + i), dev)
        need = lib.hopm_workspace_bytes(desc)
        ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
        st = torch.zeros(32, dtype=torch.uint8, device=dev)
        keep += [x, ws, st]
        c = Call(lib.hopm_iterate, desc, x.data_ptr(), 1, (ws.data_ptr() + 255) & ~255, need,
                 st.data_ptr(), sh)
        hopm_calls.append((f"hopm_sweep_{len(s)}d_{s[0]}", c, sweep_bytes(s, 4)))

    ops = [(lbl, c, b) for (lbl, c, b, _) in tvc_calls] + hopm_calls
    step_bytes = sum(b for _, _, b in ops)

    # ------------------------------------------------------------ timed steps
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        for _, c, _ in ops:
            c()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in ops] for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for s in range(args.steps):
        for j, (_, c, _) in enumerate(ops):
            ev[s][j][0].record(stream)
            c()
            ev[s][j][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    ms_per_step = total_ms / args.steps
    value = step_bytes / (ms_per_step * 1e-3) / 1e9

    per_op = {}
    for j, (lbl, _, b) in enumerate(ops):
        ms = [ev[s][j][0].elapsed_time(ev[s][j][1]) for s in range(args.steps)]
        med = statistics.median(ms)
        per_op[lbl] = {"ms_median": round(med, 4), "ms_mean": round(statistics.mean(ms), 4),
                       "GBps": round(b / (med * 1e-3) / 1e9, 1),
                       "pct_peak": round(100 * b / (med * 1e-3) / 1e9 / PEAK_HBM_GBS, 1)}
    log(json.dumps(per_op))

    # dominant kernel: the column-strip contraction kernel with the LDS
    # output window (float32, 16-byte loads, 4 waves per workgroup, 4 column
    # units per lane) that tvc_contract launches for the 32^6 modes 0-2
    dom = [(lbl, b) for (lbl, _, b, p) in tvc_calls
           if p["family"] == "col" and p["vec"] and p["window"] and p["strip_units"] == 4]
    dom_ms, dom_b = [], []
    for lbl, b in dom:
        j = [o[0] for o in ops].index(lbl)
        dom_ms += [ev[s][j][0].elapsed_time(ev[s][j][1]) for s in range(args.steps)]
        dom_b += [b] * args.steps
    avg_ms = statistics.mean(dom_ms)
    avg_b = statistics.mean(dom_b)
    achieved = avg_b / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": measured_traffic(),
                "kernel": "tvc::k_colw<1, true, 0, 4, 4, true> (float32 column strips, LDS output window)",
                "launches_per_step": len(dom), "avg_launch_ms": round(avg_ms, 4),
                "avg_bytes_per_launch": int(avg_b)}

    modes_pct = [per_op[lbl]["pct_peak"] for (lbl, _, _, _) in tvc_calls]
    extra = {
        "step_bytes": step_bytes,
        "wall_s_timed": round(wall, 3),
        "per_op": per_op,
        "tvc_pct_peak_mean": round(statistics.mean(modes_pct), 1),
        "tvc_pct_peak_std": round(statistics.stdev(modes_pct), 1),
        "plans": {lbl: p for (lbl, _, _, p) in tvc_calls},
    }

    if not args.no_extras:
        extra.update(run_extras(T, Hs, planted, dev, args))
    extra["bench_wall_s"] = round(time.perf_counter() - T0, 1)

    result = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "TVC every mode + one HOPM sweep, 1024^3 and 32^6 float32 N(0,1) "
                               "(HOPM on 10*rank-1 + N(0,0.1^2))",
                   "shapes": ["1024^3", "32^6"], "pct_of_peak": round(100 * value / PEAK_HBM_GBS, 1)},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(T, extra.get("time_to_solution"))
    result["extra"] = extra
    print(json.dumps(result), flush=True)
    return 0


def timed_ms(fn, reps, warm=1):
    """Median of `reps` single calls, each bracketed by events on the current
    stream (the queue stays full, so host launch latency is not counted)."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    return median_ms(fn, reps)


class Rocblas:
    """rocBLAS (the vendor BLAS of ROCm) through ctypes: the looped
    formulation of the contraction the paper compares against (Sec. 3: a
    batch of matrix-vector products over the (u, n_k, v) view, one per
    left index), here rocblas_[sd]gemv_strided_batched_64 on torch's stream."""
    NONE, TRANS = 111, 112
    MAX_BATCH = 32768
    MAX_COLS = 1 << 20

    def __init__(self, stream_handle):
        path = "/opt/rocm/lib/librocblas.so"
        self.lib = ctypes.CDLL(path)
        h = ctypes.c_void_p()
        self._ok(self.lib.rocblas_create_handle(ctypes.byref(h)))
        self.h = h
        self._ok(self.lib.rocblas_set_stream(h, ctypes.c_void_p(stream_handle)))
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        for name in ("rocblas_sgemv_strided_batched_64", "rocblas_dgemv_strided_batched_64"):
            fn = getattr(self.lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [vp, ctypes.c_int, i64, i64, vp, vp, i64, i64, vp, i64, i64, vp, vp, i64, i64, i64]

    @staticmethod
    def _ok(st):
        if st != 0:
            # a failed launch leaves HIP's last-error state set; clear it so
            # that later calls do not report it
            try:
                ctypes.CDLL("libamdhip64.so").hipGetLastError()
            except OSError:
                pass
            raise RuntimeError(f"rocBLAS status {st}")

    def contract(self, A, x, k, y):
        """y = A x_k x as looped matrix-vector products on the (u, n_k, v) view."""
        import torch
        dims = tuple(A.shape)
        u = math.prod(dims[:k])
        n = dims[k]
        v = math.prod(dims[k + 1:])
        f64 = A.dtype == torch.float64
        one = (ctypes.c_double if f64 else ctypes.c_float)(1.0)
        zero = (ctypes.c_double if f64 else ctypes.c_float)(0.0)
        fn = self.lib.rocblas_dgemv_strided_batched_64 if f64 else self.lib.rocblas_sgemv_strided_batched_64
        eb = A.element_size()
        if v == 1:      # y[l] = sum_m A[l, m] x[m]: A is column-major n x u, transposed
            # (in launches of at most MAX_COLS columns: rocBLAS's kernel for
            # this case has one workgroup per column)
            for l0 in range(0, u, self.MAX_COLS):
                b = min(self.MAX_COLS, u - l0)
                self._ok(fn(self.h, self.TRANS, n, b, ctypes.byref(one), A.data_ptr() + l0 * n * eb, n, 0,
                            x.data_ptr(), 1, 0, ctypes.byref(zero), y.data_ptr() + l0 * eb, 1, 0, 1))
            return
        # per left index l: y_l = A_l x with A_l column-major v x n; the
        # batch goes in launches of at most MAX_BATCH matrices (the batch
        # index is a grid dimension of rocBLAS's kernels)
        for l0 in range(0, u, self.MAX_BATCH):
            b = min(self.MAX_BATCH, u - l0)
            self._ok(fn(self.h, self.NONE, v, n, ctypes.byref(one), A.data_ptr() + l0 * n * v * eb, v, n * v,
                        x.data_ptr(), 1, 0, ctypes.byref(zero), y.data_ptr() + l0 * v * eb, 1, v, b))


def run_looped(tensors, shapes, dev, reps=5):
    """Per-mode %-of-peak of the looped rocBLAS contraction beside the
    library's, on the same tensors and vectors; each output checked against
    the library's."""
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import synth
    rb = Rocblas(torch.cuda.current_stream().cuda_stream)
    out = {}
    for A, dims in zip(tensors, shapes):
        b_a = A.element_size()
        acc = torch.float64 if A.dtype == torch.float64 else torch.float32
        for k in range(len(dims)):
            x = torch.from_numpy(synth.unit_vectors([dims[k]], 300 + k)[0]).to(acc).to(dev)
            y = torch.empty(A.numel() // dims[k], dtype=acc, device=dev)
            yl = torch.empty_like(y)
            ms_n = timed_ms(lambda: tvc.contract(A, x, k, out=y), reps)
            nb = tvc_bytes(dims, k, b_a, acc.itemsize)
            rec = {"native_pct": round(100 * nb / (ms_n * 1e-3) / 1e9 / PEAK_HBM_GBS, 1),
                   "native_ms": round(ms_n, 4)}
            try:
                ms_l = timed_ms(lambda: rb.contract(A, x, k, yl), reps)
                err = float(torch.linalg.vector_norm((y - yl).double()) / torch.linalg.vector_norm(y.double()))
                rec.update({"looped_pct": round(100 * nb / (ms_l * 1e-3) / 1e9 / PEAK_HBM_GBS, 1),
                            "looped_ms": round(ms_l, 4), "rel_diff": err})
            except RuntimeError as e:
                rec["looped_error"] = str(e)
            out[f"{len(dims)}d_{dims[0]}_mode{k}"] = rec
            del y, yl
    nat = [v["native_pct"] for v in out.values()]
    loo = [v.get("looped_pct") for v in out.values()]
    return {"per_mode": out,
            "native_mean_std": [round(statistics.mean(nat), 1), round(statistics.stdev(nat), 1)],
            "looped_mean_std": [_mean(loo), _std(loo)]}


def run_focus(spec, reps, dev):
    """Repeat one operation `reps` times after two warm-up calls (for
    rocprofv3 runs): the contraction of one mode, a Gauss-Seidel or Jacobi
    sweep, or a solve from the warm start; N(0,1) tensors (planted for
    sweeps and solves) of the named shape, converted to the named format."""
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import synth
    parts = spec.split(":")
    if parts[0] == "batch":
        r = run_batch(dev)
        return {k: v for k, v in r.items() if k != "autotune"}
    op, fmt, shape = parts[0], parts[1], parts[2]
    if "^" in shape:
        n, d = (int(v) for v in shape.split("^"))
        dims = (n,) * d
    else:
        dims = tuple(int(v) for v in shape.split("x"))
    n = dims[0]
    A, a = synth.device_planted(dims, 10.0, 0.1, 200, dev, dtype=torch.float64 if fmt == "f64" else None)
    S = None
    if fmt not in ("f32", "f64"):
        A, S = tvc.quantize(A, fmt)
    torch.cuda.synchronize()
    if op == "tvc":
        k = int(parts[3])
        acc = torch.float64 if fmt == "f64" else torch.float32
        x = torch.from_numpy(synth.unit_vectors([dims[k]], 300 + k)[0]).to(acc).to(dev)
        y = torch.empty(A.numel() // dims[k], dtype=acc, device=dev)
        fn = lambda: tvc.contract(A, x, k, out=y, scale=S)   # noqa: E731
        nbytes = tvc_bytes(dims, k, A.element_size(), acc.itemsize)
    else:
        x = tvc.pack_vectors(synth.warm_start(a, 0.9, 400), dev)
        if op == "sweep":
            fn = lambda: tvc.hopm_iterate(A, x, 1, scale=S)   # noqa: E731
            nbytes = sweep_bytes(dims, A.element_size())
        elif op == "jacobi":
            fn = lambda: tvc.hopm_jacobi_iterate(A, x, 1, scale=S)   # noqa: E731
            nbytes = math.prod(dims) * A.element_size() + 8 * sum(dims)
        else:
            x0 = x.clone()

            def fn():
                x.copy_(x0)
                tvc.hopm_solve(A, x, tol=1e-6, max_sweeps=500, scale=S)
            nbytes = 0
    ms = timed_ms(fn, reps, warm=2)
    return {"spec": spec, "reps": reps, "ms_median": round(ms, 4),
            "pct_peak": round(100 * nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 1) if nbytes else None}


def run_fp64(dev, reps=5):
    """float64 storage at the benchmark shapes (8.6 GB each): contraction in
    every mode and one HOPM sweep, % of peak (the paper's Tables 2 and 3 are
    float64)."""
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import synth
    out = {}
    for i, dims in enumerate(SHAPES):
        A = synth.device_normal(dims, 700 + i, dev, dtype=torch.float64)
        per = {}
        for k in range(len(dims)):
            x = torch.from_numpy(synth.unit_vectors([dims[k]], 300 + k)[0]).to(dev)
            y = torch.empty(A.numel() // dims[k], dtype=torch.float64, device=dev)
            ms = timed_ms(lambda: tvc.contract(A, x, k, out=y), reps)
            per[f"mode{k}"] = round(100 * tvc_bytes(dims, k, 8, 8) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 1)
            del y
        x = tvc.pack_vectors(synth.unit_vectors(dims, 60), dev)
        ms = timed_ms(lambda: tvc.hopm_iterate(A, x, 1), reps)
        vals = list(per.values())
        out[f"{len(dims)}d_{dims[0]}"] = {"tvc_pct_per_mode": per, "tvc_pct_mean": round(statistics.mean(vals), 1),
                                          "tvc_pct_std": round(statistics.stdev(vals), 1),
                                          "sweep_ms": round(ms, 3),
                                          "sweep_pct": round(100 * sweep_bytes(dims, 8) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 1)}
        del A
        torch.cuda.empty_cache()
    return out


def run_probe(src, dev):
    """The library's read and copy probes (contiguous range per workgroup,
    nontemporal 16-byte accesses): the best of several grid sizes is the
    achievable rate the contraction kernels are also set against."""
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import _lib as L
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    sink = torch.empty(64 * cus, dtype=torch.float32, device=dev)
    reads = {}
    for g in (cus, 2 * cus, 4 * cus, 8 * cus, 16 * cus):
        ms = timed_ms(lambda: tvc.probe_read(src, sink, grid=g), 10)
        reads[g] = src.numel() * src.element_size() / (ms * 1e-3) / 1e9
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    ms = timed_ms(lambda: tvc.probe_copy(a, b), 10)
    cp = 2 * a.numel() * 4 / (ms * 1e-3) / 1e9
    del a, b
    best = max(reads.values())
    return {"read_GBps": round(best, 1), "read_pct_peak": round(100 * best / PEAK_HBM_GBS, 1),
            "read_GBps_by_grid": {str(g): round(v, 1) for g, v in reads.items()},
            "copy_GBps": round(cp, 1), "bytes_read": src.numel() * src.element_size()}


def oracle_solve(A, x0, tol, workers=16):
    """The float64 oracle's Gauss-Seidel HOPM (multilinear form) from the
    exact host copy of A and the same start vectors."""
    from oracle import hopm as H
    Ah = A.cpu().numpy()
    t0 = time.perf_counter()
    ref = H.hopm(Ah, x0, tol=tol, max_sweeps=500, form="kron", workers=workers)
    return ref, time.perf_counter() - t0


def run_tts(Hs, planted, dev, tol=1e-6, reps=3):
    """Time to solution (delta < tol, one readback per sweep) from the same
    warm start (overlap 0.9 with the planted vectors), for every storage
    format, bf16 followed by float32 refinement to the same tol, and Jacobi
    sweeps; each result's lambda and vector error against the float64
    oracle's solution from the same start on the original float32 data
    (computed outside the timed region)."""
    import numpy as np
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import synth
    tts = {}
    for i, (A, s) in enumerate(zip(Hs, SHAPES)):
        x0 = synth.warm_start(planted[i], 0.9, 400 + i)
        ref, oracle_s = oracle_solve(A, x0, tol)
        stores = {"f32": (A, None)}
        for fmt in ("bf16", "f16", "e4m3"):
            stores[fmt] = tvc.quantize(A, fmt)
        runs = [("f32", "f32", None, "gs"), ("bf16", "bf16", None, "gs"), ("f16", "f16", None, "gs"),
                ("e4m3", "e4m3", None, "gs"), ("bf16+f32refine", "bf16", A, "gs"),
                ("f32_jacobi", "f32", None, "jacobi"), ("bf16_jacobi", "bf16", None, "jacobi")]
        res = {}
        for label, fmt, refine, method in runs:
            Aq, S = stores[fmt]
            times = []
            for _ in range(reps):
                x = tvc.pack_vectors(x0, dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if method == "jacobi":
                    r = tvc.hopm_jacobi_solve(Aq, x, tol=tol, max_sweeps=1000, scale=S)
                else:
                    r = tvc.hopm_solve(Aq, x, tol=tol, max_sweeps=500, check_every=1, scale=S,
                                       A_refine=refine, refine_sweeps=100 if refine is not None else 0)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            got = np.split(x.cpu().numpy(), np.cumsum(s)[:-1])
            verr = max(min(np.linalg.norm(g - e), np.linalg.norm(g + e)) for g, e in zip(got, ref.xs))
            res[label] = {"seconds": round(statistics.median(times), 5), "sweeps": r.sweeps,
                          "refine_sweeps": r.refine_sweeps, "status": r.status, "delta": r.delta,
                          "lambda": r.lam, "lambda_rel_err_vs_oracle": abs(r.lam - ref.lam) / ref.lam,
                          "vector_err_vs_oracle": float(verr),
                          "min_overlap_planted": round(min(abs(float(g @ a)) for g, a in zip(got, planted[i])), 6)}
        f32 = res["f32"]["seconds"]
        res["speedup_vs_f32"] = {k: round(f32 / v["seconds"], 3) for k, v in res.items() if k != "f32"}
        res["oracle"] = {"lambda": ref.lam, "sweeps": ref.sweeps, "seconds": round(oracle_s, 2),
                         "form": "multilinear, float64, 16 threads"}
        tts[f"{len(s)}d_{s[0]}"] = res
        log(json.dumps({f"{len(s)}d_{s[0]}": {lbl: [v["seconds"], v["sweeps"], v["refine_sweeps"], v["status"],
                                                     v["lambda_rel_err_vs_oracle"]]
                                               for lbl, v in res.items() if "refine_sweeps" in v},
                        "speedup_vs_f32": res["speedup_vs_f32"], "oracle": res["oracle"]}))
        del stores
    return tts


def run_extras(T, Hs, planted, dev, args):
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import synth

    out = {}
    out["probe"] = run_probe(T[0], dev)
    log(json.dumps(out["probe"]))
    ach = out["probe"]["read_GBps"]

    # narrow storage: every-mode contraction in bf16, fp16 and E4M3 (+ slab scales)
    ebytes = {"bf16": 2, "f16": 2, "e4m3": 1}
    for fmt, b in ebytes.items():
        res = {}
        for i, (A, s) in enumerate(zip(T, SHAPES)):
            Aq, S = tvc.quantize(A, fmt)
            for k in range(len(s)):
                x = torch.from_numpy(synth.unit_vectors([s[k]], 300 + k)[0]).float().to(dev)
                y = torch.empty(A.numel() // s[k], dtype=torch.float32, device=dev)
                ms = timed_ms(lambda: tvc.contract(Aq, x, k, out=y, scale=S), 10)
                gbs = tvc_bytes(s, k, b) / (ms * 1e-3) / 1e9
                res[f"{len(s)}d_{s[0]}_mode{k}"] = {"ms": round(ms, 4), "GBps": round(gbs, 1),
                                                    "pct_peak": round(100 * gbs / PEAK_HBM_GBS, 1),
                                                    "pct_of_probe": round(100 * gbs / ach, 1)}
            del Aq, S
        out[f"{fmt}_tvc"] = res
        log(json.dumps({fmt: res}))

    out["f64"] = run_fp64(dev)
    log(json.dumps({"f64": out["f64"]}))
    out["looped_rocblas"] = run_looped(T, SHAPES, dev)
    log(json.dumps({"looped": out["looped_rocblas"]}))
    out["time_to_solution"] = run_tts(Hs, planted, dev)
    out["derivatives_256_4"] = run_derivatives(dev)
    out["batch"] = run_batch(dev)
    if not args.no_table1:
        out["table1"] = run_table1(dev)
        out["table1_f64"] = run_table1(dev, dtype="f64")
    return out


TABLE1 = {2: 30623, 3: 979, 4: 175, 5: 63, 6: 31, 7: 19, 8: 13, 9: 10, 10: 8}


def median_ms(fn, reps, e0=None, e1=None):
    """Median over reps back-to-back calls of each call's time between two
    events around it (a single slow call, such as a clock or page-table
    hiccup, does not move it; the queue stays full, so host launch latency
    is not counted)."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return statistics.median(a.elapsed_time(b) for a, b in ev)


def _mean(v):
    v = [x for x in v if x is not None]
    return round(statistics.mean(v), 1) if v else None


def _std(v):
    v = [x for x in v if x is not None]
    return round(statistics.stdev(v), 1) if len(v) > 1 else None


def run_table1(dev, reps: int = 5, dtype: str = "f32"):
    """The paper's Table 1 hypersquare tensors (dims chosen not to be
    multiples of the vector length), in float32 (3.3-4.3 GB) or in float64,
    the paper's own precision and sizes (6.6-8.6 GB): %-of-peak of the contraction in every mode, natively and
    as looped rocBLAS matrix-vector products, and of one HOPM sweep (median
    of `reps` timed calls each), with mean and unbiased std over the modes
    (the Table 2 statistic); the canonical HOPM sweep and the one-pass
    Jacobi sweep on the same tensor."""
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import synth

    rb = Rocblas(torch.cuda.current_stream().cuda_stream)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    eb = 8 if dtype == "f64" else 4
    out = {}
    for d, n in TABLE1.items():
        dims = (n,) * d
        A = synth.device_normal(dims, 40 + d, dev, dtype=tdt)
        per, loo = [], []
        for k in range(d):
            x = torch.from_numpy(synth.unit_vectors([n], 50 + k)[0]).to(tdt).to(dev)
            y = torch.empty(A.numel() // n, dtype=tdt, device=dev)
            ms = timed_ms(lambda: tvc.contract(A, x, k, out=y), reps)
            per.append(100 * tvc_bytes(dims, k, eb, eb) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS)
            try:
                ms = timed_ms(lambda: rb.contract(A, x, k, y), reps)
                loo.append(100 * tvc_bytes(dims, k, eb, eb) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS)
            except RuntimeError:
                loo.append(None)
            del y
        x = tvc.pack_vectors(synth.unit_vectors(dims, 60), dev)
        ms = timed_ms(lambda: tvc.hopm_iterate(A, x, 1), reps)
        sweep = 100 * sweep_bytes(dims, eb) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS
        jms = timed_ms(lambda: tvc.hopm_jacobi_iterate(A, x, 1), reps)
        jac = 100 * (math.prod(dims) * eb + 8 * sum(dims)) / (jms * 1e-3) / 1e9 / PEAK_HBM_GBS
        # The canonical HOPM sweep of Sec. 3 on the same kernels: x_j is the
        # contraction of A with every other vector, one mode at a time (the
        # last modes first, so mode indices stay valid), then normalised;
        # Gauss-Seidel order.  It streams A d times, against twice for the
        # fused sweep.
        xs = [torch.from_numpy(v).to(tdt).to(dev) for v in synth.unit_vectors(dims, 60)]

        def canonical():
            for j in range(d):
                T = A
                for i in reversed(range(d)):
                    if i != j:
                        T = tvc.contract(T, xs[i], i)
                xs[j] = T / torch.linalg.vector_norm(T)

        cms = timed_ms(canonical, 5, warm=2)
        out[f"{n}^{d}"] = {"tvc_pct_mean": round(statistics.mean(per), 1),
                           "tvc_pct_std": round(statistics.stdev(per), 1) if d > 1 else 0.0,
                           "tvc_pct_per_mode": [round(p, 1) for p in per],
                           "looped_pct_mean": _mean(loo),
                           "looped_pct_std": _std(loo),
                           "looped_pct_per_mode": [None if p is None else round(p, 1) for p in loo],
                           "sweep_ms": round(ms, 3), "sweep_pct": round(sweep, 1),
                           "jacobi_sweep_ms": round(jms, 3), "jacobi_sweep_pct": round(jac, 1),
                           "canonical_sweep_ms": round(cms, 3),
                           "fused_sweep_speedup": round(cms / ms, 2)}
        log(json.dumps({f"{n}^{d}": out[f"{n}^{d}"]}))
        del A, x, xs
        torch.cuda.empty_cache()
    allp = [p for v in out.values() for p in v["tvc_pct_per_mode"]]
    alll = [p for v in out.values() for p in v["looped_pct_per_mode"]]
    out["summary"] = {"tvc_pct_mean_std_all_modes": [round(statistics.mean(allp), 1), round(statistics.stdev(allp), 1)],
                      "looped_pct_mean_std_all_modes": [_mean(alll), _std(alll)],
                      "sweep_pct_mean": round(statistics.mean(v["sweep_pct"] for v in out.values()), 1)}
    return out


def run_derivatives(dev, K: int = 10):
    """Backward of the contraction in every mode and the gradient through K
    unrolled HOPM sweeps on a 256^4 float32 tensor (17.2 GB)."""
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import autograd as AG
    from paper_2501_03121_amd import synth

    dims = (256, 256, 256, 256)
    n = math.prod(dims)
    A = synth.device_normal(dims, 500, dev)
    out = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    for k in range(4):
        g = synth.device_normal((n // dims[k],), 600 + k, dev)
        x = torch.from_numpy(synth.unit_vectors([dims[k]], 700 + k)[0]).float().to(dev)
        tvc.backward_x(A, g, k)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            tvc.backward_x(A, g, k)
        e1.record()
        torch.cuda.synchronize()
        msx = e0.elapsed_time(e1) / reps
        dA = torch.empty_like(A)
        tvc.backward_A(g, x, k, dims, out=dA)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            tvc.backward_A(g, x, k, dims, out=dA)
        e1.record()
        torch.cuda.synchronize()
        msa = e0.elapsed_time(e1) / reps
        bx = n * 4 + (n // dims[k]) * 4
        ba = n * 4 + (n // dims[k]) * 4
        out[f"mode{k}"] = {"dx_ms": round(msx, 3), "dx_GBps": round(bx / (msx * 1e-3) / 1e9, 1),
                           "dA_ms": round(msa, 3), "dA_GBps": round(ba / (msa * 1e-3) / 1e9, 1)}
        del dA, g
    Ar = A.requires_grad_(True)
    x0 = [torch.from_numpy(v).to(dev) for v in synth.unit_vectors(dims, 800)]
    times = []
    for _ in range(2):
        Ar.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam = AG.hopm(Ar, K, *x0)[0]
        loss = -lam * lam
        loss.backward()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    # passes over A: 2 per forward sweep, 2 per backward step (d steps per
    # sweep), plus reading A and writing dA once in the rank update
    passes = 2 * K + 2 * K * 4
    traffic = passes * n * 4 + 2 * n * 4
    t = min(times)
    out["unrolled_hopm_grad"] = {"sweeps": K, "seconds": round(t, 4), "passes_over_A": passes,
                                 "GBps": round(traffic / t / 1e9, 1), "lambda": float(lam)}
    log(json.dumps(out))
    del Ar, A
    torch.cuda.empty_cache()
    return out


def run_batch(dev, count: int = 512, sweeps: int = 50):
    """512 planted HOPM instances (order 3-5, dims per instance recipe, N(0,1)
    + lambda a o b o ..., lambda ~ U[2, 20]) swept 50 times by one persistent
    launch replayed from a graph; tiles and grid picked by the autotuner."""
    import torch

    import paper_2501_03121_amd as tvc
    from paper_2501_03121_amd import batch as B
    from paper_2501_03121_amd import synth

    specs = synth.batch_instances(count, 900)
    As, init = [], []
    for i, (dims, lam) in enumerate(specs):
        A = synth.device_normal(dims, 1000 + i, dev)
        vecs = synth.unit_vectors(dims, 3000 + i, "normal")
        outer = torch.ones((), dtype=torch.float64, device=dev)
        for v in vecs:
            outer = torch.tensordot(outer, torch.as_tensor(v, device=dev), dims=0)
        A.add_(outer.float(), alpha=lam)
        As.append(A)
        init.append(tvc.pack_vectors(synth.unit_vectors(dims, 5000 + i), dev))
    xs = [v.clone() for v in init]

    def reset():
        for x, v in zip(xs, init):
            x.copy_(v)

    total = sum(A.numel() for A in As)
    te, grid, table = B.autotune(As, xs, sweeps, reset, tile_choices=(1 << 18, 1 << 19, 1 << 20),
                                 grid_per_cu=(4, 8), reps=1)
    bp = B.prepare(As, xs, sweeps, tile_elems=te, grid=grid)
    g = B.capture(bp, reset)
    times = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    err = B.error_word(bp)
    res = B.results(bp)
    prof = B.profile(bp)
    t = min(times)
    nbytes = 2 * total * 4 * sweeps
    out = {"instances": count, "sweeps": sweeps, "elements": total, "tensor_GB": round(total * 4 / 1e9, 3),
           "seconds": round(t, 4), "GBps": round(nbytes / t / 1e9, 1),
           "pct_peak": round(100 * nbytes / t / 1e9 / PEAK_HBM_GBS, 1), "tile_elems": te, "grid": grid,
           "error_word": err, "degenerate": sum(r.status != 0 for r in res),
           "work_items": prof["items"], "grid_busy_fraction": round(prof["busy_fraction"], 3),
           "grid_seconds_per_phase": {k: round(v, 4) for k, v in prof["phase_s"].items()},
           "autotune": table}
    log(json.dumps({k: v for k, v in out.items() if k != "autotune"}))
    return out


def _host_info():
    import numpy as np
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        blas = [{k: d.get(k) for k in ("internal_api", "version", "num_threads", "threading_layer")}
                for d in threadpool_info() if d.get("user_api") == "blas"]
    except Exception:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "numpy": np.__version__, "blas": blas}


def cpu_baseline(tensors, tts=None, budget_s: float = 10.0):
    """The float64 oracle (NumPy) on the host: the contractions of the
    benchmark step (every mode of the 1024^3 and 32^6 tensors) from the exact
    upcast of the device bytes (upcast not timed), repeated for about
    `budget_s` seconds with all BLAS threads and again with one thread.

    `value` counts the same algorithmic bytes as the GPU figure (4 bytes per
    float32 element of A, so the two rates compare work done); the float64
    bytes the oracle actually reads (8 per element) are reported beside it.
    The oracle's HOPM time per sweep comes from the time-to-solution leg."""
    import numpy as np

    from oracle import tvc as O
    from paper_2501_03121_amd import synth
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    log("cpu baseline: copying tensors to host")
    hosts = [A.cpu().numpy().astype(np.float64) for A in tensors]

    def leg(budget):
        # the nine contractions in turn until the budget is spent (at least one)
        t, elems, calls = 0.0, 0, 0
        work = [(A, k) for A in hosts for k in range(A.ndim)]
        while t < budget and calls < 50 * len(work):
            A, k = work[calls % len(work)]
            x = synth.unit_vectors([A.shape[k]], 300 + k)[0]
            t0 = time.perf_counter()
            O.tvc(A, x, k)
            t += time.perf_counter() - t0
            elems += A.size
            calls += 1
        return t, elems, calls

    t, elems, reps = leg(budget_s)
    one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1, user_api="blas"):
            t1, e1, _ = leg(budget_s)
        one = {"value": round(e1 * 4 / t1 / 1e9, 2), "fp64_read_GBps": round(e1 * 8 / t1 / 1e9, 2),
               "cores": 1, "seconds": round(t1, 1), "elements": int(e1)}
    del hosts
    out = {"value": round(elems * 4 / t / 1e9, 2), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
           "sample": f"float64 NumPy oracle: every-mode contraction of the 1024^3 and 32^6 tensors, "
                     f"{reps} contraction(s) in turn, {t:.1f} s; value counts 4 bytes per "
                     f"element (the float32 workload's algorithmic bytes), fp64_read_GBps the 8 bytes "
                     f"per element the oracle reads",
           "fp64_read_GBps": round(elems * 8 / t / 1e9, 2), "one_thread": one, "host": _host_info()}
    if tts:
        out["oracle_hopm_seconds_per_sweep"] = {
            k: round(v["oracle"]["seconds"] / max(1, v["oracle"]["sweeps"]), 3) for k, v in tts.items()}
    return out


if __name__ == "__main__":
    sys.exit(main())
