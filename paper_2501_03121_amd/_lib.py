"""ctypes binding of libtvc.so (argument marshalling only).

Every computation runs in the HIP library; this module turns torch tensors
into the plain pointers, sizes and stream handles of the C ABI declared in
include/tvc.h.  If the shared library is missing the import of any compute
entry point fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, Structure, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint32, c_void_p
from pathlib import Path

import os

# TVC_LIBRARY overrides the library path (e.g. to compare builds).
LIB_PATH = Path(os.environ.get("TVC_LIBRARY") or Path(__file__).resolve().parent / "lib" / "libtvc.so")

TVC_OK, TVC_EINVAL, TVC_EDTYPE, TVC_EALIAS, TVC_EWORKSPACE, TVC_EHIP, TVC_EDEGENERATE, TVC_ENOTCONVERGED = range(8)
TVC_F64, TVC_F32, TVC_F16, TVC_BF16, TVC_F8E4M3 = range(5)
TVC_MAX_ORDER = 16
TVC_QUANT_TRUNCATE = 1

STATUS_NAMES = {
    TVC_OK: "TVC_OK", TVC_EINVAL: "TVC_EINVAL", TVC_EDTYPE: "TVC_EDTYPE",
    TVC_EALIAS: "TVC_EALIAS", TVC_EWORKSPACE: "TVC_EWORKSPACE", TVC_EHIP: "TVC_EHIP",
    TVC_EDEGENERATE: "TVC_EDEGENERATE", TVC_ENOTCONVERGED: "TVC_ENOTCONVERGED",
}


class TvcTensor(Structure):
    _fields_ = [
        ("order", c_int32),
        ("dtype", c_int32),
        ("dims", c_int64 * TVC_MAX_ORDER),
        ("data", c_void_p),
        ("slab_scale", c_void_p),
    ]


class HopmStats(Structure):
    _fields_ = [
        ("lam", c_double),
        ("delta", c_double),
        ("sweeps", c_int32),
        ("status", c_int32),
        ("refine_sweeps", c_int32),
        ("reserved", c_int32),
    ]


class HopmBatchDesc(Structure):
    _fields_ = [
        ("A", c_void_p),
        ("x", c_void_p),
        ("dims", c_int64 * 8),
        ("order", c_int32),
        ("tile_rows1", c_int32),
        ("tile_rows2", c_int32),
        ("nt1", c_int32),
        ("nt2", c_int32),
        ("reserved", c_int32),
        ("ws_offset", c_int64),
        ("init_slot", c_int64),
    ]


class HopmBatchPlan(Structure):
    _fields_ = [
        ("queue_slots", c_int64),
        ("initial_items", c_int64),
        ("ws_bytes", c_size_t),
        ("count", c_int32),
        ("sweeps", c_int32),
    ]


class TvcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# (name, restype, argtypes) of every C entry point the binding uses.
SIGNATURES = {
    "tvc_status_string": (c_char_p, [c_int32]),
    "tvc_last_error": (c_char_p, []),
    "tvc_version": (c_int32, []),
    "tvc_contract_workspace_bytes": (c_size_t, [POINTER(TvcTensor), c_int32]),
    "tvc_contract": (c_int32, [POINTER(TvcTensor), c_int32, c_void_p, c_void_p, c_double, c_double,
                               c_void_p, c_size_t, c_void_p]),
    "tvc_contract_noalloc_max_scratch": (c_size_t, []),
    "tvc_contract_noalloc": (c_int32, [POINTER(TvcTensor), c_int32, c_void_p, c_void_p, c_double,
                                       c_double, c_void_p]),
    "tvc_contract_plan": (c_int32, [POINTER(TvcTensor), c_int32, POINTER(c_int32), c_int32]),
    "hopm_workspace_bytes": (c_size_t, [POINTER(TvcTensor)]),
    "hopm_iterate": (c_int32, [POINTER(TvcTensor), c_void_p, c_int32, c_void_p, c_size_t, c_void_p,
                               c_void_p]),
    "hopm_solve": (c_int32, [POINTER(TvcTensor), POINTER(TvcTensor), c_void_p, c_double, c_int32,
                             c_int32, c_int32, c_void_p, c_size_t, POINTER(HopmStats), c_void_p]),
    "hopm_jacobi_iterate": (c_int32, [POINTER(TvcTensor), c_void_p, c_int32, c_void_p, c_size_t, c_void_p,
                                      c_void_p]),
    "hopm_jacobi_solve": (c_int32, [POINTER(TvcTensor), c_void_p, c_double, c_int32, c_int32, c_void_p,
                                    c_size_t, POINTER(HopmStats), c_void_p]),
    "tvc_quantize": (c_int32, [POINTER(TvcTensor), c_void_p, c_int32, c_void_p, c_int32, c_void_p]),
    "tvc_backward_x_workspace_bytes": (c_size_t, [POINTER(TvcTensor), c_int32]),
    "tvc_backward_x": (c_int32, [POINTER(TvcTensor), c_int32, c_void_p, c_void_p, c_void_p, c_size_t,
                                 c_void_p]),
    "tvc_backward_A": (c_int32, [c_int32, POINTER(c_int64), c_int32, c_int32, c_void_p, c_void_p,
                                 c_void_p, c_double, c_double, c_void_p]),
    "tvc_leave_one_out": (c_int32, [POINTER(TvcTensor), c_void_p, c_uint32, c_void_p, c_void_p, c_size_t,
                                    c_void_p]),
    "tvc_rank_update_workspace_bytes": (c_size_t, [c_int32, POINTER(c_int64), c_int32]),
    "tvc_rank_update": (c_int32, [c_int32, POINTER(c_int64), c_int32, c_void_p, c_double, c_int32,
                                  c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "hopm_iterate_record": (c_int32, [POINTER(TvcTensor), c_void_p, c_int32, c_void_p, c_size_t, c_void_p,
                                      c_void_p, c_void_p]),
    "hopm_backward_workspace_bytes": (c_size_t, [POINTER(TvcTensor), c_int32]),
    "hopm_backward": (c_int32, [POINTER(TvcTensor), c_void_p, c_void_p, c_int32, c_void_p, c_double,
                                c_double, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "hopm_batch_prepare": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p]),
    "hopm_batch_run": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_size_t, c_void_p, c_void_p]),
    "hopm_batch_error": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "hopm_batch_profile": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "tvc_set_tuning": (c_int32, [c_int32, c_int32, c_int32]),
    "tvc_probe_read": (c_int32, [c_void_p, c_size_t, c_void_p, c_int32, c_void_p]),
    "tvc_probe_copy": (c_int32, [c_void_p, c_void_p, c_size_t, c_int32, c_void_p]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libtvc.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        handle = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int) -> None:
    if status != TVC_OK:
        msg = lib().tvc_last_error().decode(errors="replace")
        raise TvcError(status, msg)


def make_tensor(order: int, dims, dtype: int, data_ptr: int, scale_ptr: int | None = None) -> TvcTensor:
    t = TvcTensor()
    t.order = order
    t.dtype = dtype
    for i, n in enumerate(dims):
        t.dims[i] = int(n)
    t.data = data_ptr
    t.slab_scale = scale_ptr if scale_ptr else None
    return t


__all__ = [
    "lib", "check", "make_tensor", "TvcTensor", "HopmStats", "HopmBatchDesc", "TvcError",
    "SIGNATURES", "LIB_PATH", "c_uint32",
]
