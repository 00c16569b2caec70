"""Torch-facing wrappers of the C ABI: tensors in, tensors out.

PyTorch supplies device memory and the current stream; every step of the
contraction, the HOPM sweep and the conversions runs in libtvc's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass

import ctypes

import torch

from . import _lib as L

_TORCH_TO_CODE = {
    torch.float64: L.TVC_F64,
    torch.float32: L.TVC_F32,
    torch.float16: L.TVC_F16,
    torch.bfloat16: L.TVC_BF16,
    torch.float8_e4m3fn: L.TVC_F8E4M3,
}
_CODE_NAMES = {L.TVC_F64: "f64", L.TVC_F32: "f32", L.TVC_F16: "f16", L.TVC_BF16: "bf16",
               L.TVC_F8E4M3: "e4m3"}
_NAME_TO_TORCH = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16,
                  "bf16": torch.bfloat16, "e4m3": torch.float8_e4m3fn}


def dtype_code(t: torch.Tensor) -> int:
    try:
        return _TORCH_TO_CODE[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported tensor dtype {t.dtype}") from None


def acc_dtype(code: int) -> torch.dtype:
    return torch.float64 if code == L.TVC_F64 else torch.float32


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _require_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on a HIP device")
        if t is not None and not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def describe(A: torch.Tensor, scale: torch.Tensor | None = None) -> L.TvcTensor:
    """C descriptor of a dense tensor (scale: per mode-0 slice, E4M3 only)."""
    _require_cuda(A, scale)
    code = dtype_code(A)
    if code == L.TVC_F8E4M3 and scale is None:
        raise ValueError("an E4M3 tensor needs its slab scales")
    if scale is not None and scale.dtype != torch.float32:
        raise TypeError("slab scales must be float32")
    return L.make_tensor(A.dim(), tuple(A.shape), code, A.data_ptr(),
                         scale.data_ptr() if scale is not None else None)


class _Workspace:
    """Per (device, stream) scratch buffer, grown on demand by torch."""

    def __init__(self):
        self._bufs: dict = {}

    def get(self, nbytes: int, device: torch.device) -> torch.Tensor | None:
        if nbytes == 0:
            return None
        key = (device.index, _stream())
        buf = self._bufs.get(key)
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
            self._bufs[key] = buf
        return buf

    @staticmethod
    def ptr(buf: torch.Tensor | None) -> int | None:
        if buf is None:
            return None
        p = buf.data_ptr()
        return (p + 255) & ~255


_WS = _Workspace()


def contract(A: torch.Tensor, x: torch.Tensor, mode: int, alpha: float = 1.0, beta: float = 0.0,
             out: torch.Tensor | None = None, scale: torch.Tensor | None = None) -> torch.Tensor:
    """Y = alpha * (A x_mode x) + beta * out (Sec. 3, Eq. (1)).

    x and the result are float64 for a float64 A, float32 otherwise.
    """
    desc = describe(A, scale)
    acc = acc_dtype(desc.dtype)
    _require_cuda(x, out)
    if x.dtype != acc or x.dim() != 1:
        raise TypeError(f"x must be a 1-D {acc} tensor")
    if not 0 <= mode < A.dim():
        raise ValueError(f"mode {mode} outside [0, {A.dim()})")
    oshape = tuple(n for i, n in enumerate(A.shape) if i != mode)
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty(oshape, dtype=acc, device=A.device)
    elif out.dtype != acc or out.numel() != A.numel() // A.shape[mode]:
        raise TypeError("out has the wrong dtype or size")
    lib = L.lib()
    need = lib.tvc_contract_workspace_bytes(desc, mode)
    ws = _WS.get(need, A.device)
    L.check(lib.tvc_contract(desc, mode, x.data_ptr(), out.data_ptr(), float(alpha), float(beta),
                             _WS.ptr(ws), int(need), _stream()))
    return out


_FAMILY = {0: "row", 1: "col", 2: "slab", 3: "stage"}


def contract_plan(A: torch.Tensor, mode: int, scale: torch.Tensor | None = None) -> dict:
    """Which kernel tvc_contract(A, mode) launches, and with what shape."""
    import ctypes
    desc = describe(A, scale)
    info = (ctypes.c_int32 * 12)()
    L.check(L.lib().tvc_contract_plan(desc, mode, info, 12))
    return {"family": _FAMILY[info[0]], "vec": bool(info[1]), "split_m": info[2],
            "nsplit": info[3], "grid": info[4], "lanes_per_row": info[5], "tail": info[6],
            "units_per_row": info[7], "window": bool(info[8]), "strip_units": info[9],
            "row_rotation": bool(info[10]), "stage_slabs": info[11]}


@dataclass
class HopmResult:
    lam: float
    delta: float
    sweeps: int
    refine_sweeps: int
    status: int


def pack_vectors(xs, device) -> torch.Tensor:
    """x_0..x_{d-1} back to back as one float64 device buffer."""
    return torch.cat([torch.as_tensor(v, dtype=torch.float64).reshape(-1) for v in xs]).to(device)


def unpack_vectors(buf: torch.Tensor, dims) -> list:
    out, o = [], 0
    for n in dims:
        out.append(buf[o:o + n])
        o += n
    return out


def hopm_workspace(A: torch.Tensor, scale: torch.Tensor | None = None) -> torch.Tensor:
    desc = describe(A, scale)
    need = L.lib().hopm_workspace_bytes(desc)
    return torch.empty(int(need) + 256, dtype=torch.uint8, device=A.device)


def hopm_iterate(A: torch.Tensor, x: torch.Tensor, sweeps: int = 1, scale: torch.Tensor | None = None,
                 ws: torch.Tensor | None = None, stats: torch.Tensor | None = None) -> torch.Tensor:
    """Run `sweeps` HOPM sweeps in place on the packed float64 vectors `x`.

    Returns the device stats record as a 32-byte uint8 tensor (see
    `read_stats`).  No host synchronisation.
    """
    desc = describe(A, scale)
    _require_cuda(x)
    if x.dtype != torch.float64 or x.numel() != sum(A.shape):
        raise TypeError("x must be float64 with sum(dims) elements")
    lib = L.lib()
    need = lib.hopm_workspace_bytes(desc)
    if ws is None:
        ws = _WS.get(need, A.device)
    if stats is None:
        # the library's first step writes every field of the record
        stats = torch.empty(32, dtype=torch.uint8, device=A.device)
    L.check(lib.hopm_iterate(desc, x.data_ptr(), int(sweeps), _WS.ptr(ws), int(need),
                             stats.data_ptr(), _stream()))
    return stats


def hopm_jacobi_iterate(A: torch.Tensor, x: torch.Tensor, sweeps: int = 1,
                        scale: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                        stats: torch.Tensor | None = None) -> torch.Tensor:
    """`sweeps` Jacobi HOPM sweeps (one pass over A each) in place on the
    packed float64 vectors `x`; returns the device stats record."""
    desc = describe(A, scale)
    _require_cuda(x)
    if x.dtype != torch.float64 or x.numel() != sum(A.shape):
        raise TypeError("x must be float64 with sum(dims) elements")
    lib = L.lib()
    need = lib.hopm_workspace_bytes(desc)
    if ws is None:
        ws = _WS.get(need, A.device)
    if stats is None:
        # the library's first step writes every field of the record
        stats = torch.empty(32, dtype=torch.uint8, device=A.device)
    L.check(lib.hopm_jacobi_iterate(desc, x.data_ptr(), int(sweeps), _WS.ptr(ws), int(need),
                                    stats.data_ptr(), _stream()))
    return stats


def hopm_jacobi_solve(A: torch.Tensor, x: torch.Tensor, tol: float = 1e-6, max_sweeps: int = 1000,
                      check_every: int = 1, scale: torch.Tensor | None = None) -> HopmResult:
    """Jacobi sweeps until delta < tol or max_sweeps (synchronises every
    check_every sweeps)."""
    desc = describe(A, scale)
    _require_cuda(x)
    lib = L.lib()
    need = lib.hopm_workspace_bytes(desc)
    ws = _WS.get(need, A.device)
    hp = _pinned_stats()
    st = lib.hopm_jacobi_solve(desc, x.data_ptr(), float(tol), int(max_sweeps), int(check_every),
                               _WS.ptr(ws), int(need), hp, _stream())
    h = L.HopmStats.from_buffer_copy(ctypes.string_at(_PINNED_STATS.data_ptr(), ctypes.sizeof(L.HopmStats)))
    if st not in (L.TVC_OK, L.TVC_ENOTCONVERGED):
        L.check(st)
    return HopmResult(h.lam, h.delta, h.sweeps, h.refine_sweeps, st)


def _pinned_stats():
    """The result record in pinned host memory: the library reads each
    convergence check straight into it."""
    global _PINNED_STATS
    if _PINNED_STATS is None:
        _PINNED_STATS = torch.empty(ctypes.sizeof(L.HopmStats), dtype=torch.uint8, pin_memory=True)
    return ctypes.cast(_PINNED_STATS.data_ptr(), ctypes.POINTER(L.HopmStats))


def read_stats(stats: torch.Tensor) -> HopmResult:
    raw = stats.cpu().numpy().tobytes()
    s = L.HopmStats.from_buffer_copy(raw)
    return HopmResult(s.lam, s.delta, s.sweeps, s.refine_sweeps, s.status)


def hopm_solve(A: torch.Tensor, x: torch.Tensor, tol: float = 1e-6, max_sweeps: int = 1000,
               check_every: int = 1, scale: torch.Tensor | None = None,
               A_refine: torch.Tensor | None = None, refine_sweeps: int = 0,
               raise_on_nonconvergence: bool = False) -> HopmResult:
    """Sweep until delta < tol or max_sweeps; then optional float32
    refinement sweeps on A_refine.  Synchronises every check_every sweeps."""
    desc = describe(A, scale)
    _require_cuda(x)
    rdesc = describe(A_refine) if A_refine is not None else None
    lib = L.lib()
    need = lib.hopm_workspace_bytes(desc)
    ws = _WS.get(need, A.device)
    hp = _pinned_stats()
    st = lib.hopm_solve(desc, rdesc, x.data_ptr(), float(tol), int(max_sweeps), int(check_every),
                        int(refine_sweeps), _WS.ptr(ws), int(need), hp, _stream())
    h = L.HopmStats.from_buffer_copy(ctypes.string_at(_PINNED_STATS.data_ptr(), ctypes.sizeof(L.HopmStats)))
    if st not in (L.TVC_OK, L.TVC_ENOTCONVERGED) or (st == L.TVC_ENOTCONVERGED and raise_on_nonconvergence):
        L.check(st)
    return HopmResult(h.lam, h.delta, h.sweeps, h.refine_sweeps, st)


_PINNED_STATS = None


def quantize(A32: torch.Tensor, fmt: str, truncate: bool = False):
    """Convert a float32 tensor to 'f16', 'bf16' or 'e4m3' storage.

    Returns (stored tensor, slab scales or None)."""
    desc = describe(A32)
    if desc.dtype != L.TVC_F32:
        raise TypeError("quantize needs a float32 tensor")
    tdt = _NAME_TO_TORCH[fmt]
    code = _TORCH_TO_CODE[tdt]
    out = torch.empty(A32.shape, dtype=tdt, device=A32.device)
    scale = None
    if code == L.TVC_F8E4M3:
        scale = torch.empty(A32.shape[0], dtype=torch.float32, device=A32.device)
    L.check(L.lib().tvc_quantize(desc, out.data_ptr(), code,
                                 scale.data_ptr() if scale is not None else None,
                                 L.TVC_QUANT_TRUNCATE if truncate else 0, _stream()))
    return out, scale


def probe_read(buf: torch.Tensor, sink: torch.Tensor, grid: int = 0) -> None:
    _require_cuda(buf, sink)
    L.check(L.lib().tvc_probe_read(buf.data_ptr(), buf.numel() * buf.element_size(),
                                   sink.data_ptr(), int(grid), _stream()))


def probe_copy(src: torch.Tensor, dst: torch.Tensor, grid: int = 0) -> None:
    _require_cuda(src, dst)
    L.check(L.lib().tvc_probe_copy(src.data_ptr(), dst.data_ptr(), src.numel() * src.element_size(),
                                   int(grid), _stream()))


# ---------------------------------------------------------------- derivatives
def _dims_array(shape):
    import ctypes
    arr = (ctypes.c_int64 * len(shape))(*[int(n) for n in shape])
    return arr


def backward_x(A: torch.Tensor, g: torch.Tensor, mode: int, scale: torch.Tensor | None = None) -> torch.Tensor:
    """dx = A contracted with g over every mode but `mode` (one pass over A)."""
    desc = describe(A, scale)
    acc = acc_dtype(desc.dtype)
    _require_cuda(g)
    if g.dtype != acc or g.numel() != A.numel() // A.shape[mode]:
        raise TypeError("g has the wrong dtype or size")
    dx = torch.empty(A.shape[mode], dtype=acc, device=A.device)
    lib = L.lib()
    need = lib.tvc_backward_x_workspace_bytes(desc, mode)
    ws = _WS.get(need, A.device)
    L.check(lib.tvc_backward_x(desc, mode, g.data_ptr(), dx.data_ptr(), _WS.ptr(ws), int(need), _stream()))
    return dx


def backward_A(g: torch.Tensor, x: torch.Tensor, mode: int, shape, alpha: float = 1.0, beta: float = 0.0,
               out: torch.Tensor | None = None) -> torch.Tensor:
    """dA = alpha * (g outer x at `mode`) + beta * out."""
    _require_cuda(g, x, out)
    code = dtype_code(g)
    if code not in (L.TVC_F32, L.TVC_F64) or x.dtype != g.dtype:
        raise TypeError("g and x must both be float32 or both float64")
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty(tuple(shape), dtype=g.dtype, device=g.device)
    dims = _dims_array(shape)
    L.check(L.lib().tvc_backward_A(len(shape), dims, code, int(mode), g.data_ptr(), x.data_ptr(),
                                   out.data_ptr(), float(alpha), float(beta), _stream()))
    return out


def leave_one_out(A: torch.Tensor, v: torch.Tensor, modes=None, scale: torch.Tensor | None = None) -> torch.Tensor:
    """out_m = A contracted with v_k over every k != m, for m in `modes`
    (default all); v and the result are packed float64 vectors."""
    desc = describe(A, scale)
    _require_cuda(v)
    if v.dtype != torch.float64 or v.numel() != sum(A.shape):
        raise TypeError("v must be float64 with sum(dims) elements")
    mask = (1 << A.dim()) - 1 if modes is None else sum(1 << int(m) for m in modes)
    out = torch.zeros_like(v)
    lib = L.lib()
    need = lib.hopm_workspace_bytes(desc)
    ws = _WS.get(need, A.device)
    L.check(lib.tvc_leave_one_out(desc, v.data_ptr(), mask, out.data_ptr(), _WS.ptr(ws), int(need), _stream()))
    return out


def rank_update(shape, factors: torch.Tensor, coef: torch.Tensor, A: torch.Tensor | None = None,
                alpha: float = 0.0, out: torch.Tensor | None = None, dtype=torch.float32) -> torch.Tensor:
    """D = alpha * A + sum_r coef[r] * (outer product of the factor vectors of term r).

    factors: float64 (R, sum(shape)); coef: float64 (R,)."""
    _require_cuda(factors, coef, A, out)
    R = int(coef.numel())
    if out is None:
        out = torch.empty(tuple(shape), dtype=dtype, device=factors.device)
    code = dtype_code(out)
    dims = _dims_array(shape)
    lib = L.lib()
    need = lib.tvc_rank_update_workspace_bytes(len(shape), dims, R)
    ws = _WS.get(need, out.device)
    L.check(lib.tvc_rank_update(len(shape), dims, code, A.data_ptr() if A is not None else None,
                                float(alpha), R, factors.data_ptr(), coef.data_ptr(), out.data_ptr(),
                                _WS.ptr(ws), int(need), _stream()))
    return out


def hopm_iterate_record(A: torch.Tensor, x: torch.Tensor, sweeps: int, norms: torch.Tensor,
                        scale: torch.Tensor | None = None) -> torch.Tensor:
    """hopm_iterate that writes ||y|| of every (sweep, j) step into `norms`."""
    desc = describe(A, scale)
    _require_cuda(x, norms)
    if norms.dtype != torch.float64 or norms.numel() < sweeps * A.dim():
        raise TypeError("norms must be float64 with sweeps * order elements")
    lib = L.lib()
    need = lib.hopm_workspace_bytes(desc)
    ws = _WS.get(need, A.device)
    stats = torch.zeros(32, dtype=torch.uint8, device=A.device)
    L.check(lib.hopm_iterate_record(desc, x.data_ptr(), int(sweeps), _WS.ptr(ws), int(need),
                                    stats.data_ptr(), norms.data_ptr(), _stream()))
    return stats


def hopm_backward(A: torch.Tensor, xs: torch.Tensor, norms: torch.Tensor, sweeps: int,
                  gx: torch.Tensor | None, glam: float, gA_scale: float = 0.0, want_dA: bool = True,
                  want_dx0: bool = False, scale: torch.Tensor | None = None):
    """Reverse pass through `sweeps` HOPM sweeps; returns (dA or None, dx0 or None)."""
    desc = describe(A, scale)
    _require_cuda(xs, norms, gx)
    acc = acc_dtype(desc.dtype)
    dA = torch.empty(A.shape, dtype=acc, device=A.device) if want_dA else None
    dx0 = torch.empty(sum(A.shape), dtype=torch.float64, device=A.device) if want_dx0 else None
    lib = L.lib()
    need = lib.hopm_backward_workspace_bytes(desc, int(sweeps))
    ws = torch.empty(int(need) + 256, dtype=torch.uint8, device=A.device)
    L.check(lib.hopm_backward(desc, xs.data_ptr(), norms.data_ptr(), int(sweeps),
                              gx.data_ptr() if gx is not None else None, float(glam), float(gA_scale),
                              dA.data_ptr() if dA is not None else None,
                              dx0.data_ptr() if dx0 is not None else None,
                              _WS.ptr(ws), int(need), _stream()))
    return dA, dx0
