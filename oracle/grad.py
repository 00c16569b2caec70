"""Oracle for derivatives of the contraction and of unrolled HOPM (test
infrastructure only).

Adjoints of Y = A x_k x (Sec. 3 definition, (u, n_k, v) view):
  dx[m]       = sum_{l, r} A[l, m, r] * g[l, r]     (A contracted with g over
                                                     every mode but k)
  dA[l, m, r] = g[l, r] * x[m]                      (rank-1 outer product)
for an incoming gradient g of Y.

Unrolled HOPM: K canonical Gauss-Seidel sweeps (see `oracle.hopm`) from fixed
initial vectors give unit vectors u_0..u_{d-1} and lambda = ||y|| at the last
step.  With U = u_0 o ... o u_{d-1} (||U|| = 1) and lambda = <A, U>, the loss
||A - lambda U||_F^2 equals ||A||^2 - lambda^2.  Its gradient with respect to
A (the initial vectors held fixed) is taken by a hand-written reverse pass
through every (sweep, j) step: for y = A contracted with x_m (m != j) and
x_j = y / ||y||,
  ybar  = (xbar_j - x_j <x_j, xbar_j>) / ||y||  (+ the seed at the last step)
  Abar += ybar at mode j outer x_m at the other modes
  xbar_m += A contracted with ybar at mode j and x_k at the modes k != j, m.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .hopm import leave_one_out
from .tvc import matricized_dims


def tvc_grad_x(A: np.ndarray, g: np.ndarray, k: int) -> np.ndarray:
    """dx = A contracted with g over every mode except k."""
    A64 = np.asarray(A, dtype=np.float64)
    u, n, v = matricized_dims(A64.shape, k)
    g2 = np.asarray(g, dtype=np.float64).reshape(u, v)
    return np.einsum("lmr,lr->m", A64.reshape(u, n, v), g2)


def tvc_grad_A(g: np.ndarray, x: np.ndarray, k: int, dims: Sequence[int]) -> np.ndarray:
    """dA = g outer x placed at mode k (shape `dims`)."""
    u, n, v = matricized_dims(dims, k)
    g2 = np.asarray(g, dtype=np.float64).reshape(u, v)
    x64 = np.asarray(x, dtype=np.float64).reshape(n)
    return np.einsum("lr,m->lmr", g2, x64).reshape(tuple(dims))


def outer(vecs: Sequence[np.ndarray]) -> np.ndarray:
    """v_0 o v_1 o ... o v_{d-1} as a dense float64 tensor."""
    out = np.ones(())
    for v in vecs:
        out = np.multiply.outer(out, np.asarray(v, dtype=np.float64).reshape(-1))
    return out


def _forward(A64: np.ndarray, xs0: Sequence[np.ndarray], K: int):
    d = A64.ndim
    xs = [np.asarray(x, dtype=np.float64).reshape(-1).copy() for x in xs0]
    steps = []
    for _ in range(K):
        for j in range(d):
            before = [x.copy() for x in xs]
            y = leave_one_out(A64, xs, j)
            nrm = float(np.linalg.norm(y))
            xs[j] = y / nrm
            steps.append((j, before, nrm, xs[j].copy()))
    return xs, steps


def hopm_loss(A: np.ndarray, xs0: Sequence[np.ndarray], K: int) -> float:
    """L = ||A - lambda U||_F^2 after K sweeps (computed from its definition)."""
    A64 = np.asarray(A, dtype=np.float64)
    xs, steps = _forward(A64, xs0, K)
    lam = steps[-1][2]
    return float(np.sum((A64 - lam * outer(xs)) ** 2))


def hopm_loss_and_grad(A: np.ndarray, xs0: Sequence[np.ndarray], K: int):
    """(L, dL/dA, [dL/dx0_j]) for L = ||A||^2 - lambda^2 after K sweeps."""
    A64 = np.asarray(A, dtype=np.float64)
    d = A64.ndim
    xs, steps = _forward(A64, xs0, K)
    lam = steps[-1][2]
    L = float(np.sum(A64 * A64)) - lam * lam
    Abar = 2.0 * A64
    xbar = [np.zeros_like(x) for x in xs]
    for s in reversed(range(len(steps))):
        j, before, nrm, xnew = steps[s]
        xb = xbar[j]
        ybar = (xb - xnew * float(np.dot(xnew, xb))) / nrm
        if s == len(steps) - 1:
            ybar = ybar + (-2.0 * lam) * xnew      # d(-lambda^2)/dy at the last step
        xbar[j] = np.zeros_like(xb)                 # the old x_j is not used by this step
        vecs = [ybar if m == j else before[m] for m in range(d)]
        Abar += outer(vecs)
        for m in range(d):
            if m != j:
                xbar[m] = xbar[m] + leave_one_out(A64, vecs, m)
    return L, Abar, xbar
