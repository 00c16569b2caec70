"""The C ABI: the shared library loads, exports every function include/tvc.h
declares, and rejects bad arguments on the host before any device work.
CPU only (no kernel is launched)."""
import ctypes
import re
from pathlib import Path

import pytest

from paper_2501_03121_amd import _lib as L

HEADER = Path(__file__).resolve().parents[1] / "include" / "tvc.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_declares_core_calls():
    names = declared_functions()
    for n in ("tvc_contract", "hopm_iterate", "hopm_solve", "tvc_contract_workspace_bytes",
              "hopm_workspace_bytes", "tvc_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    assert set(declared_functions()) <= set(L.SIGNATURES)


def test_status_strings():
    lib = L.lib()
    for code, name in L.STATUS_NAMES.items():
        assert lib.tvc_status_string(code).decode() == name
    assert lib.tvc_version() >= 100


def tensor(dims, dtype=L.TVC_F32, data=4096, scale=None):
    return L.make_tensor(len(dims), dims, dtype, data, scale)


def test_contract_argument_errors():
    lib = L.lib()
    ok = tensor((4, 5, 6))
    x, y = 1 << 20, 2 << 20
    cases = [
        (tensor((4, 5, 6), data=0), 0, x, y, L.TVC_EINVAL),          # NULL data
        (tensor((4, 0, 6)), 0, x, y, L.TVC_EINVAL),                  # zero dim
        (tensor((4, 5, 6), data=4098), 0, x, y, L.TVC_EINVAL),       # misaligned
        (ok, 3, x, y, L.TVC_EINVAL),                                  # bad mode
        (ok, -1, x, y, L.TVC_EINVAL),
        (ok, 0, 0, y, L.TVC_EINVAL),                                  # NULL x
        (ok, 0, x, 4096 + 8, L.TVC_EALIAS),                           # y inside A
        (tensor((4, 5, 6), dtype=9), 0, x, y, L.TVC_EDTYPE),
        (tensor((4, 5, 6), dtype=L.TVC_F8E4M3), 1, x, y, L.TVC_EDTYPE),   # no scales
    ]
    for t, mode, xp, yp, want in cases:
        got = lib.tvc_contract(t, mode, xp, yp, 1.0, 0.0, None, 0, None)
        assert got == want, (mode, got, want, lib.tvc_last_error())
        assert lib.tvc_last_error()
    bad = L.make_tensor(17, (1,) * 16, L.TVC_F32, 4096)
    assert lib.tvc_contract(bad, 0, x, y, 1.0, 0.0, None, 0, None) == L.TVC_EINVAL


def test_hopm_argument_errors():
    lib = L.lib()
    st = L.HopmStats()
    one = tensor((7,))
    assert lib.hopm_iterate(one, 1 << 20, 1, 1 << 24, 1 << 20, 1 << 22, None) == L.TVC_EINVAL
    t = tensor((4, 5, 6))
    need = lib.hopm_workspace_bytes(t)
    assert need > 0
    assert lib.hopm_iterate(t, 1 << 20, 1, None, 0, 1 << 22, None) == L.TVC_EWORKSPACE
    assert lib.hopm_iterate(t, 1 << 20, 1, 1 << 24, need - 1, 1 << 22, None) == L.TVC_EWORKSPACE
    assert lib.hopm_iterate(t, 1 << 20, 0, 1 << 24, need, 1 << 22, None) == L.TVC_EINVAL
    # x overlapping A
    assert lib.hopm_iterate(t, 4096, 1, 1 << 24, need, 1 << 22, None) == L.TVC_EALIAS
    assert lib.hopm_solve(t, None, 1 << 20, 1e-6, 0, 1, 0, 1 << 24, need, st, None) == L.TVC_EINVAL
    r = tensor((4, 5, 7))
    assert lib.hopm_solve(t, r, 1 << 20, 1e-6, 5, 1, 1, 1 << 24, need, st, None) == L.TVC_EINVAL


def test_quantize_argument_errors():
    lib = L.lib()
    t = tensor((4, 5))
    assert lib.tvc_quantize(t, 1 << 20, L.TVC_F32, None, 0, None) == L.TVC_EDTYPE
    assert lib.tvc_quantize(tensor((4, 5), dtype=L.TVC_F16), 1 << 20, L.TVC_BF16, None, 0, None) == L.TVC_EDTYPE
    assert lib.tvc_quantize(t, 4096 + 16, L.TVC_BF16, None, 0, None) == L.TVC_EALIAS
    assert lib.tvc_quantize(t, 1 << 20, L.TVC_F8E4M3, None, 0, None) == L.TVC_EINVAL


def test_workspace_sizes_are_aligned_and_monotone():
    lib = L.lib()
    small = lib.hopm_workspace_bytes(tensor((16, 16, 16)))
    big = lib.hopm_workspace_bytes(tensor((64, 64, 64)))
    assert small % 256 == 0 and big % 256 == 0 and big > small
    assert lib.tvc_contract_workspace_bytes(tensor((1 << 20,)), 0) > 0   # long single row splits
    assert lib.tvc_contract_workspace_bytes(tensor((64, 64, 64)), 1) == 0


def test_batch_and_tuning_argument_errors():
    lib = L.lib()
    assert lib.hopm_batch_profile(None, 1 << 20, None) == L.TVC_EINVAL
    assert lib.hopm_batch_profile(1 << 20, None, None) == L.TVC_EINVAL
    assert lib.hopm_batch_error(None, 1 << 20, None) == L.TVC_EINVAL
    assert lib.hopm_batch_error(1 << 20, None, None) == L.TVC_EINVAL
    plan = L.HopmBatchPlan()
    descs = (L.HopmBatchDesc * 1)()
    d = descs[0]
    d.A, d.x, d.order = 1 << 20, 1 << 22, 2
    d.dims[0] = d.dims[1] = 8
    assert lib.hopm_batch_prepare(descs, 1, 5, 0, ctypes.byref(plan)) == L.TVC_EINVAL   # order < 3
    d.order, d.dims[2] = 3, 8
    assert lib.hopm_batch_prepare(descs, 0, 5, 0, ctypes.byref(plan)) == L.TVC_EINVAL   # no instances
    assert lib.hopm_batch_prepare(descs, 1, 0, 0, ctypes.byref(plan)) == L.TVC_EINVAL   # no sweeps
    assert lib.hopm_batch_prepare(descs, 1, 5, 0, ctypes.byref(plan)) == L.TVC_OK
    assert plan.queue_slots == 5 * (descs[0].nt1 + descs[0].nt2 + 2)
    assert lib.hopm_batch_run(None, ctypes.byref(plan), 0, 1 << 24, plan.ws_bytes, 1 << 22, None) == L.TVC_EINVAL
    assert lib.hopm_batch_run(1 << 20, ctypes.byref(plan), 0, 1 << 24, plan.ws_bytes - 1, 1 << 22, None) == L.TVC_EWORKSPACE
    assert lib.tvc_set_tuning(5, 0, 0) == L.TVC_EINVAL
    assert lib.tvc_set_tuning(4, 0, 0) == L.TVC_OK
    assert lib.tvc_set_tuning(1, 0, 3) == L.TVC_EINVAL
    t = tensor((64, 9, 12), dtype=L.TVC_F32)             # small slabs: staged family
    info = (ctypes.c_int32 * 8)()
    assert lib.tvc_contract_plan(t, 1, info, 8) == L.TVC_OK and info[0] == 3
    assert lib.tvc_set_tuning(3, -1, 0) == L.TVC_OK      # staged family off ...
    assert lib.tvc_contract_plan(t, 1, info, 8) == L.TVC_OK and info[0] == 2
    assert lib.tvc_set_tuning(3, 0, 0) == L.TVC_OK       # ... and on again
    assert lib.tvc_contract_plan(t, 1, info, 8) == L.TVC_OK and info[0] == 3
    assert lib.tvc_contract_plan(t, 1, None, 8) == L.TVC_EINVAL
    t = tensor((32,) * 6, dtype=L.TVC_F32)               # short columns: output window
    info = (ctypes.c_int32 * 9)()
    assert lib.tvc_contract_plan(t, 2, info, 9) == L.TVC_OK and info[0] == 1 and info[8] == 1
    assert lib.tvc_set_tuning(1, 0, -1) == L.TVC_OK      # window off ...
    assert lib.tvc_contract_plan(t, 2, info, 9) == L.TVC_OK and info[8] == 0
    assert lib.tvc_set_tuning(1, 0, 0) == L.TVC_OK       # ... and on again
    assert lib.tvc_contract_plan(t, 2, info, 9) == L.TVC_OK and info[8] == 1
    t = tensor((64, 1024, 1024), dtype=L.TVC_F32)        # long columns: direct stores
    assert lib.tvc_contract_plan(t, 1, info, 9) == L.TVC_OK and info[0] == 1 and info[8] == 0


# The staged kernel copies blocks of whole slabs into an LDS buffer (32 KB;
# 64 KB with the output window for 4- and 8-byte elements) whose end holds
# the M weights (accumulator type, 16-byte aligned), and loads a block with
# 16-byte vectors; with the output window (64 KB for 4- and 8-byte elements,
# else 8 KB) a block's outputs take at most half of it.  The planner's block sizes must
# keep all of that in bounds, for every format and many slab shapes.
def test_staged_blocks_fit_their_lds():
    import itertools
    eb = {L.TVC_F64: 8, L.TVC_F32: 4, L.TVC_F16: 2, L.TVC_BF16: 2, L.TVC_F8E4M3: 1}
    ab = {L.TVC_F64: 8, L.TVC_F32: 4, L.TVC_F16: 4, L.TVC_BF16: 4, L.TVC_F8E4M3: 4}
    shapes = [(n,) * d for n, d in ((31, 6), (19, 7), (13, 8), (10, 9), (8, 10))]
    shapes += [(40, m, r) for m, r in itertools.product((1, 3, 8, 37, 150, 300, 600, 1300, 2000),
                                                       (1, 2, 3, 4, 5, 7, 8, 12, 13, 20, 31, 32))]
    shapes += [(300000, 9, 13), (64, 9, 12), (3000, 91, 1), (600, 5, 8), (700, 3, 4)]
    seen = 0
    for dims in shapes:
        for dt in eb:
            scale = (1 << 21) if dt == L.TVC_F8E4M3 else None
            t = tensor(dims, dtype=dt, data=1 << 20, scale=scale)
            for k in range(len(dims)):
                info = (ctypes.c_int32 * 12)()
                assert L.lib().tvc_contract_plan(t, k, info, 12) == L.TVC_OK
                if info[0] != 3:
                    assert info[11] == 0
                    continue
                seen += 1
                M = dims[k]
                R = 1
                for n in dims[k + 1:]:
                    R *= n
                sb = info[11]
                block = sb * M * R * eb[dt]
                wres = (M * ab[dt] + 15) // 16 * 16
                assert sb >= 1 and block % 16 == 0, (dims, dt, k, sb)
                wide = eb[dt] >= 4 and info[8]
                assert block + wres <= (65536 if wide else 32768), (dims, dt, k, sb, block, wres)
                if info[8]:
                    assert sb * R * ab[dt] <= (32768 if wide else 4096), (dims, dt, k, sb)
    assert seen > 100


# The planner's choices on the benchmark and Table 1 shapes for a 256-CU
# part (the count the library assumes without a device), as measured on the
# MI355X: the width of the windowed column strips by row pitch, M and
# format, and where small slabs are staged.  (family, window, units per lane
# of the strips, row rotation, staged slabs > 0)
PLAN_CASES = [
    ((32,) * 6, 1, L.TVC_F32, ("col", 1, 4, 1, False)),    # 4 MB rows: 4 units, rotated
    ((32,) * 6, 0, L.TVC_F32, ("col", 1, 2, 0, False)),    # 128 MB rows, M >= 32: 2
    ((32,) * 6, 3, L.TVC_F32, ("col", 1, 2, 0, False)),    # 4 KB rows: 2
    ((32,) * 6, 4, L.TVC_F32, ("slab", 1, 0, 0, False)),
    ((32,) * 6, 5, L.TVC_F32, ("row", 1, 0, 0, False)),
    ((63,) * 5, 0, L.TVC_F32, ("col", 1, 2, 0, False)),    # odd pitch, M >= 32: 2
    ((63,) * 5, 0, L.TVC_F64, ("col", 1, 4, 1, False)),    # float64, not a multiple of 4 KB: 4
    ((10,) * 9, 0, L.TVC_F32, ("col", 1, 1, 0, False)),    # M < 32: 1
    ((10,) * 9, 7, L.TVC_F32, ("stage", 1, 0, 0, True)),
    ((8,) * 10, 8, L.TVC_F32, ("stage", 1, 0, 0, True)),   # 2-unit slab rows
    ((8,) * 10, 8, L.TVC_F64, ("stage", 1, 0, 0, True)),   # 4-unit rows, float64 only
    ((16,) * 7, 5, L.TVC_F32, ("slab", 1, 0, 0, False)),   # 4-unit rows, float32: slab kernel
    ((32,) * 6, 4, L.TVC_F8E4M3, ("stage", 1, 0, 0, True)),
]


def test_plans_of_benchmark_and_table1_shapes():
    fam = ("row", "col", "slab", "stage")
    for dims, k, dt, want in PLAN_CASES:
        scale = (1 << 21) if dt == L.TVC_F8E4M3 else None
        t = tensor(dims, dtype=dt, data=1 << 20, scale=scale)
        info = (ctypes.c_int32 * 12)()
        assert L.lib().tvc_contract_plan(t, k, info, 12) == L.TVC_OK
        got = (fam[info[0]], info[8], info[9], info[10], info[11] > 0)
        assert got == want, (dims, k, dt, got, want)
