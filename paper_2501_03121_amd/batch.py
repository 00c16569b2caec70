"""Batched HOPM: planning, launch, graph capture and autotuning.

The planner orders the instances largest first (so the longest chains of
dependent phases start first), lets hopm_batch_prepare size the work items
and the workspace, and keeps every buffer the launch needs.  The autotuner
times the persistent launch for candidate tile sizes and grid sizes on the
actual batch and keeps the fastest, with a JSON cache keyed by a coarse
signature of the batch.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
import time
from dataclasses import dataclass, field

import torch

from . import _lib as L
from . import core


@dataclass
class BatchPlan:
    dims: list                     # dims per instance, in the caller's order
    order: list                    # instance index of each slot (largest first)
    descs: object                  # host ctypes array of hopm_batch_desc
    d_descs: torch.Tensor          # device copy of descs
    plan: L.HopmBatchPlan
    ws: torch.Tensor
    stats: torch.Tensor            # count * 32 bytes, device
    err: torch.Tensor              # one uint32, device
    tile_elems: int
    grid: int
    keep: list = field(default_factory=list)


def signature(dims_list, sweeps) -> str:
    tot = sum(math.prod(d) for d in dims_list)
    orders = sorted({len(d) for d in dims_list})
    return f"n{len(dims_list)}_s{sweeps}_o{'-'.join(map(str, orders))}_e{int(math.log2(max(tot, 1)))}"


def prepare(As, xs, sweeps: int, tile_elems: int = 1 << 16, grid: int = 0) -> BatchPlan:
    """As: float32 device tensors (order >= 3); xs: packed float64 device
    vectors of each instance (updated in place by every run)."""
    if len(As) != len(xs) or not As:
        raise ValueError("need one vector buffer per tensor")
    n = len(As)
    sizes = [A.numel() for A in As]
    order = sorted(range(n), key=lambda i: -sizes[i])
    descs = (L.HopmBatchDesc * n)()
    for slot, i in enumerate(order):
        A, x = As[i], xs[i]
        if A.dtype != torch.float32 or not A.is_cuda or not A.is_contiguous():
            raise TypeError("batch tensors must be contiguous float32 device tensors")
        if x.dtype != torch.float64 or x.numel() != sum(A.shape):
            raise TypeError("batch vectors must be float64 with sum(dims) elements")
        d = descs[slot]
        d.A = A.data_ptr()
        d.x = x.data_ptr()
        for m, nm in enumerate(A.shape):
            d.dims[m] = int(nm)
        d.order = A.dim()
        d.tile_rows1 = 0
        d.tile_rows2 = 0
    plan = L.HopmBatchPlan()
    L.check(L.lib().hopm_batch_prepare(descs, n, int(sweeps), int(tile_elems), ctypes.byref(plan)))
    dev = As[0].device
    raw = bytes(descs)
    d_descs = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
    ws = torch.empty(int(plan.ws_bytes) + 256, dtype=torch.uint8, device=dev)
    stats = torch.zeros(32 * n, dtype=torch.uint8, device=dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    return BatchPlan([tuple(A.shape) for A in As], order, descs, d_descs, plan, ws, stats, err,
                     int(tile_elems), int(grid), keep=[As, xs])


def _ws_ptr(bp: BatchPlan) -> int:
    return (bp.ws.data_ptr() + 255) & ~255


def run(bp: BatchPlan) -> None:
    """Enqueue the batch (three kernels) on the current stream."""
    s = torch.cuda.current_stream().cuda_stream
    L.check(L.lib().hopm_batch_run(bp.d_descs.data_ptr(), ctypes.byref(bp.plan), int(bp.grid),
                                   _ws_ptr(bp), int(bp.plan.ws_bytes), bp.stats.data_ptr(), s))


def error_word(bp: BatchPlan) -> int:
    s = torch.cuda.current_stream().cuda_stream
    L.check(L.lib().hopm_batch_error(_ws_ptr(bp), bp.err.data_ptr(), s))
    return int(bp.err.item())


def profile(bp: BatchPlan) -> dict:
    """Work items run and the persistent grid's time split (seconds summed
    over workgroups) between waiting for queue slots and running items, for
    the last run on this plan's workspace."""
    out = torch.zeros(6, dtype=torch.int64, device=bp.ws.device)
    s = torch.cuda.current_stream().cuda_stream
    L.check(L.lib().hopm_batch_profile(_ws_ptr(bp), out.data_ptr(), s))
    items, wait, p1, s1, p2, s2 = (int(v) for v in out.cpu().tolist())
    work = p1 + s1 + p2 + s2
    return {"items": items, "wait_s": wait / 1e8, "work_s": work / 1e8,
            "phase_s": {"pass1_tiles": p1 / 1e8, "x0_x1": s1 / 1e8, "pass2_tiles": p2 / 1e8,
                        "w_chain": s2 / 1e8},
            "busy_fraction": work / max(wait + work, 1)}


def results(bp: BatchPlan) -> list:
    """Per-instance HopmResult in the caller's instance order."""
    raw = bp.stats.cpu().numpy().tobytes()
    out = [None] * len(bp.order)
    for slot, i in enumerate(bp.order):
        s = L.HopmStats.from_buffer_copy(raw[32 * slot:32 * slot + 32])
        out[i] = core.HopmResult(s.lam, s.delta, s.sweeps, s.refine_sweeps, s.status)
    return out


def capture(bp: BatchPlan, reset=None):
    """Capture one batch launch (preceded by `reset()`, e.g. restoring the
    initial vectors) in a torch CUDA graph; returns the graph."""
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        if reset is not None:
            reset()
        run(bp)            # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        if reset is not None:
            reset()
        run(bp)
    return g


def _time_once(bp: BatchPlan, reset) -> float:
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(bp)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def autotune(As, xs, sweeps: int, reset, tile_choices=(1 << 14, 1 << 15, 1 << 16, 1 << 17, 1 << 18),
             grid_per_cu=(2, 4, 8), cache_path: str | None = None, reps: int = 2):
    """Time the batch for each (tile_elems, grid) candidate; return
    (best tile_elems, best grid, table).  `reset()` must restore the initial
    vectors.  Results are cached by `signature` in `cache_path` if given."""
    key = signature([tuple(A.shape) for A in As], sweeps)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            e = cache[key]
            return e["tile_elems"], e["grid"], e.get("table", [])
    cus = torch.cuda.get_device_properties(As[0].device).multi_processor_count
    table = []
    best = None
    for te in tile_choices:
        for gpc in grid_per_cu:
            bp = prepare(As, xs, sweeps, tile_elems=te, grid=gpc * cus)
            _time_once(bp, reset)            # warm-up
            t = min(_time_once(bp, reset) for _ in range(reps))
            if error_word(bp) != 0:
                continue
            table.append({"tile_elems": te, "grid": gpc * cus, "seconds": t})
            if best is None or t < best[2]:
                best = (te, gpc * cus, t)
            del bp
    if best is None:
        raise RuntimeError("every batch configuration reported an error")
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = {"tile_elems": best[0], "grid": best[1], "table": table}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best[0], best[1], table
