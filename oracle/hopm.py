"""Oracle for the higher-order power method (test infrastructure only).

Canonical HOPM (paper, Sec. 3): given an order-d tensor A and d unit vectors
x_0..x_{d-1}, each external iteration j contracts A with every vector except
x_j (d-1 contractions, d(d-1) per sweep) and replaces x_j by the normalised
result.  The vectors are updated in place, so later j use the vectors already
updated in the same sweep (Gauss-Seidel; the reading that Algorithm 1 also
implies, because its buffer W is built from vectors refreshed in the sweep).

Readings of the paper used here (the paper gives no stopping rule and never
names the singular value):
  * lambda = ||y|| at j = d-1 before normalisation, which equals
    A x_0 x_0 ... x_{d-1} x_{d-1} after that normalisation (>= 0; the vectors
    carry the sign).
  * delta = max_j ||x_j(sweep i) - x_j(sweep i-1)||_2, tested after a sweep.
  * a zero-norm contraction result is an error (the vector cannot be scaled).

`leave_one_out_kron` gives the same vector as the multilinear form
sum_{l,r} A[l,m,r] wl[l] wr[r] on the (u, n_j, v) view with Kronecker weight
vectors (two matrix-vector products, blocked for tensors too large to upcast
whole); `hopm(..., form="kron")` uses it for tensors of 10^9 elements and more.

`jacobi_hopm` is the Jacobi variant (every vector of a sweep from the previous
sweep's vectors), which the paper does not use; it is the oracle of the
library's one-pass Jacobi sweep.

`dhopm3` follows Algorithm 1 (dHOPM_3) at one process: three buffers, with the
buffer W carried from j to j+1 for j >= 1.  It is a schedule model, used to
check the contraction count (d-1)(d+2)/2 per sweep and that it reaches the
same vectors as the canonical form.  `m_seq` is Eq. (3).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

from .tvc import matricized_dims, tvc


class DegenerateError(ValueError):
    """A contraction result had zero norm, so the vector cannot be normalised."""


@dataclass
class HopmResult:
    xs: list                     # final unit vectors, float64
    lam: float                   # ||y|| at the last j of the last sweep
    sweeps: int                  # sweeps performed
    deltas: list = field(default_factory=list)    # delta after every sweep
    lams: list = field(default_factory=list)      # lambda after every sweep
    norms: list = field(default_factory=list)     # ||y|| at every (i, j)
    tvcs: int = 0                # contractions performed
    touched: int = 0             # streamed elements (Eq. (3) accounting)


def leave_one_out(A64: np.ndarray, xs: Sequence[np.ndarray], j: int,
                  log: list | None = None) -> np.ndarray:
    """y = A contracted with every x_m, m != j (vector of length n_j).

    Modes are contracted from the last to the first, so the position of every
    remaining mode equals its original label.  If `log` is given, one entry
    (input elements, output elements, vector length) is appended per
    contraction.
    """
    Y = A64
    for m in reversed(range(A64.ndim)):
        if m == j:
            continue
        out = tvc(Y, xs[m], m)
        if log is not None:
            log.append((Y.size, out.size, Y.shape[m]))
        Y = out
    return np.asarray(Y, dtype=np.float64).reshape(-1)


def kron(vecs: Sequence[np.ndarray]) -> np.ndarray:
    """v_0 (x) v_1 (x) ... as one flat float64 vector, the last vector varying
    fastest (the last-order layout of Sec. 3); [1.0] for an empty list."""
    out = np.ones(1)
    for v in vecs:
        out = np.multiply.outer(out, np.asarray(v, dtype=np.float64).reshape(-1)).reshape(-1)
    return out


def leave_one_out_kron(A: np.ndarray, xs: Sequence[np.ndarray], j: int,
                       block_elems: int = 1 << 26, workers: int = 1) -> np.ndarray:
    """The vector of `leave_one_out`, written as the multilinear form on the
    (u, n_j, v) view of Sec. 3:
        y[m] = sum_{l, r} A[l, m, r] * wl[l] * wr[r],
        wl = x_0 (x) ... (x) x_{j-1},   wr = x_{j+1} (x) ... (x) x_{d-1}.
    Two library matrix-vector products: the larger of l and r is contracted
    first.  For tensors too large to upcast whole, the first product runs
    over blocks of about `block_elems` elements (each block upcast exactly to
    float64 on its own) and the block results are added in block order;
    `workers` threads may compute the blocks (the order of the additions does
    not change).  A may be float32; every product is float64.
    """
    A = np.asarray(A)
    d = A.ndim
    u, n, v = matricized_dims(A.shape, j)
    wl = kron(xs[:j])
    wr = kron(xs[j + 1:])
    if v >= u:
        # z[l, m] = sum_r A[l, m, r] wr[r], over blocks of (l, m) rows
        A2 = A.reshape(u * n, v)
        rows = max(1, block_elems // v)
        starts = range(0, u * n, rows)
        parts = _map(lambda p0: np.asarray(A2[p0:p0 + rows], dtype=np.float64) @ wr, starts, workers)
        z = np.concatenate(parts)
        return wl @ z.reshape(u, n)
    # z[m, r] = sum_l wl[l] A[l, m, r], over blocks of l
    A2 = A.reshape(u, n * v)
    rows = max(1, block_elems // (n * v))
    starts = range(0, u, rows)
    parts = _map(lambda l0: wl[l0:l0 + rows] @ np.asarray(A2[l0:l0 + rows], dtype=np.float64),
                 starts, workers)
    z = np.zeros(n * v, dtype=np.float64)
    for p in parts:
        z += p
    return z.reshape(n, v) @ wr


def _map(fn, items, workers: int) -> list:
    """[fn(i) for i in items], on `workers` threads when workers > 1."""
    if workers <= 1:
        return [fn(i) for i in items]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items))


def _touched(log: list, nvec: int) -> int:
    # Eq. (3) accounting: every contraction reads its input tensor and its
    # vector and writes its output; the normalisation touches 3 n elements.
    return sum(i + o + v for (i, o, v) in log) + 3 * nvec


def hopm(A: np.ndarray, xs0: Sequence[np.ndarray], sweeps: int | None = None,
         tol: float | None = None, max_sweeps: int = 1000, form: str = "chain",
         workers: int = 1) -> HopmResult:
    """Canonical Gauss-Seidel HOPM in float64.

    Runs `sweeps` sweeps, or, if `sweeps` is None, until delta < tol or
    `max_sweeps` sweeps.  form = "chain" forms each leave-one-out vector by
    d - 1 contractions (`leave_one_out`); form = "kron" by the multilinear
    form of `leave_one_out_kron` (the same vector, for tensors whose chain of
    contractions would be slow on the host; A is then upcast block by block
    on `workers` threads and may stay float32).
    """
    if form == "kron":
        return _hopm_kron(A, xs0, sweeps, tol, max_sweeps, workers)
    A64 = np.asarray(A, dtype=np.float64)
    d = A64.ndim
    if d < 2:
        raise ValueError("HOPM needs order >= 2")
    xs = [np.asarray(x, dtype=np.float64).reshape(-1).copy() for x in xs0]
    for j in range(d):
        if xs[j].shape[0] != A64.shape[j]:
            raise ValueError(f"x_{j} has length {xs[j].shape[0]}, mode size {A64.shape[j]}")
    res = HopmResult(xs=xs, lam=0.0, sweeps=0)
    limit = sweeps if sweeps is not None else max_sweeps
    for _ in range(limit):
        old = [x.copy() for x in xs]
        for j in range(d):
            log: list = []
            y = leave_one_out(A64, xs, j, log)
            nrm = float(np.linalg.norm(y))
            if nrm == 0.0:
                raise DegenerateError(f"zero-norm contraction at j={j}")
            xs[j] = y / nrm
            res.norms.append(nrm)
            res.tvcs += len(log)
            res.touched += _touched(log, A64.shape[j])
        res.lam = res.norms[-1]
        res.sweeps += 1
        delta = max(float(np.linalg.norm(xs[j] - old[j])) for j in range(d))
        res.deltas.append(delta)
        res.lams.append(res.lam)
        if sweeps is None and tol is not None and delta < tol:
            break
    res.xs = xs
    return res


def _hopm_kron(A: np.ndarray, xs0: Sequence[np.ndarray], sweeps: int | None,
               tol: float | None, max_sweeps: int, workers: int = 1) -> HopmResult:
    """`hopm` with each leave-one-out vector from `leave_one_out_kron`."""
    A = np.asarray(A)
    d = A.ndim
    if d < 2:
        raise ValueError("HOPM needs order >= 2")
    xs = [np.asarray(x, dtype=np.float64).reshape(-1).copy() for x in xs0]
    res = HopmResult(xs=xs, lam=0.0, sweeps=0)
    limit = sweeps if sweeps is not None else max_sweeps
    for _ in range(limit):
        old = [x.copy() for x in xs]
        for j in range(d):
            y = leave_one_out_kron(A, xs, j, workers=workers)
            nrm = float(np.linalg.norm(y))
            if nrm == 0.0:
                raise DegenerateError(f"zero-norm contraction at j={j}")
            xs[j] = y / nrm
            res.norms.append(nrm)
        res.lam = res.norms[-1]
        res.sweeps += 1
        delta = max(float(np.linalg.norm(xs[j] - old[j])) for j in range(d))
        res.deltas.append(delta)
        res.lams.append(res.lam)
        if sweeps is None and tol is not None and delta < tol:
            break
    res.xs = xs
    return res


def jacobi_hopm(A: np.ndarray, xs0: Sequence[np.ndarray], sweeps: int | None = None,
                tol: float | None = None, max_sweeps: int = 1000, form: str = "chain",
                workers: int = 1) -> HopmResult:
    """Jacobi variant of HOPM in float64 (not the paper's sweep, which is
    Gauss-Seidel): in every sweep, y_j = A contracted with x_m for every
    m != j is formed for all j from the vectors of the PREVIOUS sweep, and
    only then x_j = s_j y_j / ||y_j|| with s_j = -1 when <y_j, x_j(old)> < 0,
    else 1 (reading: the sign keeps each vector's orientation from sweep to
    sweep; the directions are those of the plain Jacobi iteration, and
    without it the signs of an even-order iteration can alternate forever).
    lambda = ||y_{d-1}||, delta as in `hopm`.  form / workers as in `hopm`.
    """
    A = np.asarray(A)
    d = A.ndim
    if d < 2:
        raise ValueError("HOPM needs order >= 2")
    A64 = np.asarray(A, dtype=np.float64) if form == "chain" else A
    xs = [np.asarray(x, dtype=np.float64).reshape(-1).copy() for x in xs0]
    res = HopmResult(xs=xs, lam=0.0, sweeps=0)
    limit = sweeps if sweeps is not None else max_sweeps
    for _ in range(limit):
        old = [x.copy() for x in xs]
        if form == "kron":
            ys = [leave_one_out_kron(A64, old, j, workers=workers) for j in range(d)]
        else:
            ys = [leave_one_out(A64, old, j) for j in range(d)]
        for j in range(d):
            nrm = float(np.linalg.norm(ys[j]))
            if nrm == 0.0:
                raise DegenerateError(f"zero-norm contraction at j={j}")
            sign = -1.0 if float(np.dot(ys[j], old[j])) < 0.0 else 1.0
            xs[j] = sign * ys[j] / nrm
            res.norms.append(nrm)
        res.lam = res.norms[-1]
        res.sweeps += 1
        delta = max(float(np.linalg.norm(xs[j] - old[j])) for j in range(d))
        res.deltas.append(delta)
        res.lams.append(res.lam)
        if sweeps is None and tol is not None and delta < tol:
            break
    res.xs = xs
    return res


def dhopm3(A: np.ndarray, xs0: Sequence[np.ndarray], sweeps: int) -> HopmResult:
    """Algorithm 1 (dHOPM_3) at one process, as a schedule model in float64.

    For external iteration j the first contraction is
      j = 0:  W = A x_1 x_1               (remaining modes 0, 2, 3, ...)
      j = 1:  W = A x_0 x_0               (remaining modes 1, 2, ...)
      j >= 2: W = W x_{j-1} x_{j-1}       (W from j-1; remaining j, j+1, ...)
    followed by the contractions of the trailing modes above max(1, j), each
    on the previous result.  Mode labels are the original ones of A (reading
    of the paper: the mode subscripts of Algorithm 1 name modes of A, not
    positions in the shrinking intermediate).
    """
    A64 = np.asarray(A, dtype=np.float64)
    d = A64.ndim
    if d < 2:
        raise ValueError("HOPM needs order >= 2")
    xs = [np.asarray(x, dtype=np.float64).reshape(-1).copy() for x in xs0]
    res = HopmResult(xs=xs, lam=0.0, sweeps=0)
    for _ in range(sweeps):
        old = [x.copy() for x in xs]
        W = None
        W_modes: list = []
        for j in range(d):
            log: list = []
            if j == 0:
                src, src_modes, first = A64, list(range(d)), 1
            elif j == 1:
                src, src_modes, first = A64, list(range(d)), 0
            else:
                src, src_modes, first = W, W_modes, j - 1
            pos = src_modes.index(first)
            Y = tvc(src, xs[first], pos)
            log.append((src.size, Y.size, src.shape[pos]))
            modes = [m for m in src_modes if m != first]
            if j >= 1:
                W, W_modes = Y, list(modes)
            # trailing modes above max(1, j), contracted in increasing order
            for m in range(max(1, j) + 1, d):
                pos = modes.index(m)
                out = tvc(Y, xs[m], pos)
                log.append((Y.size, out.size, Y.shape[pos]))
                Y = out
                modes.pop(pos)
            y = np.asarray(Y, dtype=np.float64).reshape(-1)
            nrm = float(np.linalg.norm(y))
            if nrm == 0.0:
                raise DegenerateError(f"zero-norm contraction at j={j}")
            xs[j] = y / nrm
            res.norms.append(nrm)
            res.tvcs += len(log)
            res.touched += _touched(log, A64.shape[j])
        res.lam = res.norms[-1]
        res.sweeps += 1
        res.deltas.append(max(float(np.linalg.norm(xs[j] - old[j])) for j in range(d)))
        res.lams.append(res.lam)
    res.xs = xs
    return res


def m_seq(n: int, d: int) -> int:
    """Eq. (3): streamed elements of one external iteration of canonical HOPM
    on a hypersquare n^d tensor: the tensor, the intermediates written and
    read back, and the vectors plus normalisation."""
    return n ** d + 2 * sum(n ** k for k in range(2, d)) + (d + 3) * n


def streamed_ratio(n: int, d: int) -> float:
    """H^{-1} at one process: canonical streamed elements per sweep divided by
    those of Algorithm 1, both counted with the Eq. (3) accounting."""
    canon = d * m_seq(n, d)
    return canon / dhopm3_touched(n, d)


def dhopm3_touched(n: int, d: int) -> int:
    """Streamed elements of one Algorithm 1 sweep on a hypersquare n^d tensor,
    counted like Eq. (3) (each contraction reads input and vector and writes
    output; each normalisation touches 3 n), from the schedule of `dhopm3`."""
    total = 0
    for j in range(d):
        # first contraction
        src = n ** d if j < 2 else n ** (d - j + 1)
        out = src // n
        total += src + out + n
        # trailing contractions above max(1, j)
        size = out
        for _ in range(max(1, j) + 1, d):
            total += size + size // n + n
            size //= n
        total += 3 * n
    return total


def tvcs_per_sweep_dhopm3(d: int) -> int:
    """Contractions per Algorithm 1 sweep: 2 (d-1) for j = 0, 1 plus d - j for
    every j >= 2; the paper states the saving over d(d-1) as (d-1)(d-2)/2."""
    return 2 * (d - 1) + sum(d - j for j in range(2, d))
