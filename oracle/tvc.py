"""Oracle for the k-mode tensor-vector contraction (test infrastructure only).

Definition (paper, Sec. 3 "Background"): a dense order-d tensor A with mode
sizes n_0..n_{d-1} is stored last-order (C row-major), zero-based.  The k-mode
contraction with a vector x of length n_k gives Y = A x_k x, a tensor with the
d-1 remaining modes in their original order.  Sec. 3 also views A as the
matrix A^{uv x n_k} with u = prod_{i<k} n_i and v = prod_{i>k} n_i, so that
    Y[l, r] = sum_m A[l, m, r] * x[m],   l < u, m < n_k, r < v.
The BLAS-like scaling of Eq. (1) is Y := alpha * (A x_k x) + beta * Y, where
beta == 0 means Y is not read (reading of the paper: ordinary BLAS rules).

All arithmetic is float64 on the exact upcast of the stored values.
"""
from __future__ import annotations

import itertools
from typing import Sequence

import numpy as np


def matricized_dims(dims: Sequence[int], k: int) -> tuple[int, int, int]:
    """(u, n_k, v) of Sec. 3: u = product of the modes before k, v = after k."""
    d = len(dims)
    if not 0 <= k < d:
        raise ValueError(f"mode {k} out of range for order {d}")
    u = int(np.prod(dims[:k], dtype=np.int64)) if k > 0 else 1
    v = int(np.prod(dims[k + 1:], dtype=np.int64)) if k < d - 1 else 1
    return u, int(dims[k]), v


def output_dims(dims: Sequence[int], k: int) -> tuple[int, ...]:
    """Modes of Y = A x_k x: mode k removed, the others kept in order (Sec. 3)."""
    return tuple(int(n) for i, n in enumerate(dims) if i != k)


def tvc(A: np.ndarray, x: np.ndarray, k: int, alpha: float = 1.0,
        beta: float = 0.0, y: np.ndarray | None = None) -> np.ndarray:
    """Y = alpha * (A x_k x) + beta * Y in float64 (Sec. 3 and Eq. (1)).

    A is any real array (upcast exactly to float64), x has length n_k.  The
    contraction is one library product on the (u, n_k, v) view (a stack of u
    vector-matrix products x^T A[l]); no blocking or reordering beyond that.
    """
    A64 = np.asarray(A, dtype=np.float64)
    x64 = np.asarray(x, dtype=np.float64).reshape(-1)
    dims = A64.shape
    u, n, v = matricized_dims(dims, k)
    if x64.shape[0] != n:
        raise ValueError(f"x has length {x64.shape[0]}, mode {k} has size {n}")
    A3 = A64.reshape(u, n, v)
    # one stacked vector-matrix product: for every l, x^T A[l, :, :]
    out = np.matmul(x64, A3)
    out = float(alpha) * out
    if beta != 0.0:
        if y is None:
            raise ValueError("beta != 0 needs y")
        out = out + float(beta) * np.asarray(y, dtype=np.float64).reshape(u, v)
    return out.reshape(output_dims(dims, k))


def tvc_loops(A: np.ndarray, x: np.ndarray, k: int) -> np.ndarray:
    """Brute-force TVC: one Python loop per output element and per summand.

    Written straight from the index definition of Sec. 3 with full
    multi-indices (no matricized view), for tiny tensors only.
    """
    A64 = np.asarray(A, dtype=np.float64)
    x64 = np.asarray(x, dtype=np.float64).reshape(-1)
    dims = A64.shape
    odims = output_dims(dims, k)
    Y = np.zeros(odims, dtype=np.float64)
    for oidx in itertools.product(*[range(n) for n in odims]):
        s = 0.0
        for m in range(dims[k]):
            full = oidx[:k] + (m,) + oidx[k:]
            s += float(A64[full]) * float(x64[m])
        Y[oidx] = s
    return Y


def contract_all(A: np.ndarray, xs: Sequence[np.ndarray], order: Sequence[int]) -> float:
    """Contract every mode of A, one mode at a time, in the given mode order.

    Modes are named by their original labels; after each contraction the
    position of a later mode shifts down by the number of modes removed
    before it.  The result is the scalar A x_0 x_0 ... x_{d-1} x_{d-1}.
    """
    Y = np.asarray(A, dtype=np.float64)
    remaining = list(range(Y.ndim))
    for mode in order:
        pos = remaining.index(mode)
        Y = tvc(Y, xs[mode], pos)
        remaining.pop(pos)
    return float(np.asarray(Y).reshape(()))


def tvc_sample(A: np.ndarray, x: np.ndarray, k: int, lr: np.ndarray) -> np.ndarray:
    """Selected outputs Y[l, r] of the (u, n_k, v) view, each computed alone.

    Intended for tensors too large to contract whole in float64: for every
    requested (l, r) the fiber A[l, :, r] is gathered, upcast exactly to
    float64 and dotted with x.  `lr` is an integer array of shape (S, 2).
    """
    dims = A.shape
    u, n, v = matricized_dims(dims, k)
    A3 = A.reshape(u, n, v)
    x64 = np.asarray(x, dtype=np.float64).reshape(-1)
    lr = np.asarray(lr, dtype=np.int64).reshape(-1, 2)
    out = np.empty(lr.shape[0], dtype=np.float64)
    for s, (l, r) in enumerate(lr):
        fiber = np.asarray(A3[l, :, r], dtype=np.float64)
        out[s] = float(np.dot(fiber, x64))
    return out


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """Norm-wise relative error ||got - ref||_2 / ||ref||_2 (0 if both are 0)."""
    g = np.asarray(got, dtype=np.float64).reshape(-1)
    r = np.asarray(ref, dtype=np.float64).reshape(-1)
    den = float(np.linalg.norm(r))
    num = float(np.linalg.norm(g - r))
    if den == 0.0:
        return num
    return num / den
