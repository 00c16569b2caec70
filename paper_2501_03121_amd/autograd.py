"""torch.autograd Functions over the HIP contraction and the HOPM sweep.

`tvc(A, x, mode)` differentiates Y = A x_mode x with the library's backward
kernels: dx = A contracted with the incoming gradient over every other mode
(one pass over A), dA = gradient outer x (write-bound).

`hopm(A, sweeps, *x0)` runs `sweeps` HOPM sweeps from the initial vectors
and returns (lambda, x_0, ..., x_{d-1}).  The forward keeps only the vectors
at sweep boundaries and the norm of every (sweep, j) step (the checkpoints);
the backward is the library's reverse pass, which rebuilds the state of each
step from those checkpoints, takes one leave-one-out contraction per step
(two passes over A) and writes dA once as a sum of rank-1 terms.
"""
from __future__ import annotations

import torch

from . import core


class TVCFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, x, mode):
        ctx.mode = int(mode)
        ctx.save_for_backward(A, x)
        return core.contract(A, x, ctx.mode)

    @staticmethod
    def backward(ctx, gy):
        A, x = ctx.saved_tensors
        g = gy.contiguous().reshape(-1)
        dA = dx = None
        if ctx.needs_input_grad[0]:
            dA = core.backward_A(g, x, ctx.mode, A.shape).to(A.dtype)
        if ctx.needs_input_grad[1]:
            dx = core.backward_x(A, g, ctx.mode)
        return dA, dx, None


def tvc(A: torch.Tensor, x: torch.Tensor, mode: int) -> torch.Tensor:
    """Differentiable A x_mode x (float32 or float64 A)."""
    return TVCFunction.apply(A, x, mode)


class HOPMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, sweeps, *x0):
        d = A.dim()
        dims = tuple(A.shape)
        x = core.pack_vectors([v.detach() for v in x0], A.device)
        xs = torch.empty((sweeps + 1, x.numel()), dtype=torch.float64, device=A.device)
        xs[0].copy_(x)
        norms = torch.empty(sweeps * d, dtype=torch.float64, device=A.device)
        for i in range(sweeps):
            core.hopm_iterate_record(A, x, 1, norms[i * d:(i + 1) * d])
            xs[i + 1].copy_(x)
        ctx.save_for_backward(A, xs, norms)
        ctx.sweeps = sweeps
        ctx.dims = dims
        ctx.x_dtypes = [v.dtype for v in x0]
        lam = norms[-1].clone()
        return (lam, *[v.clone() for v in core.unpack_vectors(xs[sweeps], dims)])

    @staticmethod
    def backward(ctx, glam, *gxs):
        A, xs, norms = ctx.saved_tensors
        dims = ctx.dims
        need_A = ctx.needs_input_grad[0]
        need_x = any(ctx.needs_input_grad[2:])
        if not (need_A or need_x):
            return (None, None) + (None,) * len(dims)
        parts = [g.reshape(-1).to(torch.float64) if g is not None
                 else torch.zeros(n, dtype=torch.float64, device=A.device) for g, n in zip(gxs, dims)]
        gx = torch.cat(parts).contiguous()
        gl = float(glam.item()) if glam is not None else 0.0
        dA, dx0 = core.hopm_backward(A, xs, norms, ctx.sweeps, gx, gl, 0.0, want_dA=need_A,
                                     want_dx0=need_x)
        if dA is not None and dA.dtype != A.dtype:
            dA = dA.to(A.dtype)
        dxs = [None] * len(dims)
        if dx0 is not None:
            dxs = [v.to(dt) for v, dt in zip(core.unpack_vectors(dx0, dims), ctx.x_dtypes)]
        return (dA, None, *dxs)


def hopm(A: torch.Tensor, sweeps: int, *x0: torch.Tensor):
    """Differentiable K-sweep HOPM: returns (lambda, x_0, ..., x_{d-1})."""
    return HOPMFunction.apply(A, int(sweeps), *x0)


def rank1_loss(A: torch.Tensor, sweeps: int, *x0: torch.Tensor) -> torch.Tensor:
    """||A - lambda u_0 o ... o u_{d-1}||_F^2 after `sweeps` sweeps, written as
    ||A||^2 - lambda^2 (the u are unit vectors and lambda = <A, U>)."""
    lam = hopm(A, sweeps, *x0)[0]
    return (A.double() * A.double()).sum() - lam * lam
