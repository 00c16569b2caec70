"""Autotuner for the contraction kernels.

For a list of (tensor, mode) workloads it times every candidate launch
configuration of the kernel families those workloads use (grid cap in
workgroups per compute unit, and wave groups per column tile for the
column-streaming family), keeps the configuration with the smallest total
time, and installs it with tvc_set_tuning.  Results can be cached in a JSON
file keyed by the workload signature.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import _lib as L
from . import core

FAMILY = {"row": 0, "col": 1, "slab": 2, "stage": 3, "hopm_strips": 4}


def set_tuning(family: str, blocks_per_cu: int = 0, split_m: int = 0) -> None:
    L.check(L.lib().tvc_set_tuning(FAMILY[family], int(blocks_per_cu), int(split_m)))


def reset() -> None:
    for f in FAMILY:
        set_tuning(f, 0, 0)


def _time(calls, reps: int) -> float:
    for c in calls:
        c()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        for c in calls:
            c()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(workloads, reps: int = 5, bpc=(2, 4, 8, 16), split=(1, 2, 4), cache_path: str | None = None):
    """workloads: list of (A, x, mode, out).  Returns {family: (bpc, split_m, ms)}."""
    key = ";".join(f"{tuple(A.shape)}:{A.dtype}:{k}" for A, _, k, _ in workloads)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            best = {fam: tuple(v) for fam, v in cache[key].items()}
            for fam, (b, s, _) in best.items():
                set_tuning(fam, b, s)
            return best
    reset()
    by_family: dict = {}
    for A, x, k, out in workloads:
        fam = core.contract_plan(A, k)["family"]
        by_family.setdefault(fam, []).append((A, x, k, out))
    best = {}
    for fam, wl in by_family.items():
        calls = [lambda A=A, x=x, k=k, out=out: core.contract(A, x, k, out=out) for A, x, k, out in wl]
        cands = itertools.product(bpc, split if fam == "col" else (0,))
        for b, s in cands:
            set_tuning(fam, b, s)
            ms = _time(calls, reps)
            if fam not in best or ms < best[fam][2]:
                best[fam] = (b, s, ms)
        set_tuning(fam, best[fam][0], best[fam][1])
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = {fam: list(v) for fam, v in best.items()}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best
