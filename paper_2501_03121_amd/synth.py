"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

Only random numbers and the construction of planted test tensors live here;
none of the contraction or power-method arithmetic does.  Host inputs use
NumPy's PCG64; device inputs use torch's seeded device generator, and any
check on them reads the exact device bytes back.

Seeds follow one convention: the tensor entries, the planted vectors, the
noise and the initial vectors use seed, seed + 1, seed + 2 and seed + 3.
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0, dtype=np.float64) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=shape).astype(dtype)


def normal(shape, seed: int, std: float = 1.0, dtype=np.float64) -> np.ndarray:
    return (std * rng(seed).standard_normal(size=shape)).astype(dtype)


def integers(shape, seed: int, lo: int, hi: int, dtype=np.float64) -> np.ndarray:
    """Integer-valued floats in [lo, hi] (sums of products stay exact)."""
    return rng(seed).integers(lo, hi + 1, size=shape).astype(dtype)


def unit_vectors(dims, seed: int, kind: str = "uniform") -> list:
    """One unit-norm float64 vector per mode (uniform[-1,1] or normal entries)."""
    g = rng(seed)
    out = []
    for n in dims:
        v = g.uniform(-1.0, 1.0, size=n) if kind == "uniform" else g.standard_normal(n)
        out.append(v / np.linalg.norm(v))
    return out


def planted_rank1(dims, lam: float, noise: float, seed: int, noise_kind: str = "uniform",
                  vec_kind: str = "uniform"):
    """lam * a_0 o a_1 o ... + noise * E on the host, float64.

    E is i.i.d. uniform[-1,1] (noise_kind "uniform") or standard normal;
    the a_k are unit vectors.  Returns (tensor, [a_k])."""
    a = unit_vectors(dims, seed + 1, vec_kind)
    T = np.ones(())
    for v in a:
        T = np.multiply.outer(T, v)
    if noise_kind == "uniform":
        E = uniform(tuple(dims), seed + 2)
    else:
        E = normal(tuple(dims), seed + 2)
    return lam * T + noise * E, a


def warm_start(a: list, overlap: float, seed: int) -> list:
    """Unit vectors with inner product `overlap` with each a_k:
    overlap * a_k + sqrt(1 - overlap^2) * g_k with g_k a unit vector
    orthogonal to a_k."""
    g = rng(seed)
    out = []
    s = math.sqrt(max(0.0, 1.0 - overlap * overlap))
    for v in a:
        r = g.standard_normal(v.shape[0])
        r -= np.dot(r, v) * v
        r /= np.linalg.norm(r)
        out.append(overlap * v + s * r)
    return out


# ---------------------------------------------------------------- device
def device_normal(shape, seed: int, device, dtype=None, std: float = 1.0):
    """N(0, std^2) entries generated on the device (torch Philox)."""
    import torch
    dtype = dtype or torch.float32
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    t = torch.empty(tuple(shape), dtype=dtype, device=device)
    t.normal_(0.0, std, generator=gen)
    return t


def device_planted(dims, lam: float, std: float, seed: int, device, dtype=None):
    """lam * a_0 o ... o a_{d-1} + N(0, std^2) built on the device slice by
    slice along mode 0; the planted unit vectors come from the host
    generator (normal entries).  Returns (tensor, [a_k] as float64 numpy)."""
    import torch
    dtype = dtype or torch.float32
    A = device_normal(dims, seed + 2, device, dtype, std)
    a = unit_vectors(dims, seed + 1, "normal")
    rest = torch.ones((), dtype=torch.float64, device=device)
    for v in a[1:]:
        rest = torch.tensordot(rest, torch.as_tensor(v, device=device), dims=0)
    rest = rest.to(dtype)
    for i in range(dims[0]):
        A[i].add_(rest, alpha=float(lam * a[0][i]))
    return A, a


def batch_instances(count: int, seed: int, orders=(3, 4, 5), lo: int = 16, hi: int = 256):
    """Shapes and planted strengths of a batch of HOPM instances.

    Order uniform in `orders`; every dim uniform in [lo, floor(hi^(3/d))]
    (at most hi^3 elements per instance); lambda ~ U[2, 20]."""
    g = rng(seed)
    out = []
    for _ in range(count):
        d = int(g.choice(orders))
        top = int(math.floor(hi ** (3.0 / d) + 1e-9))
        dims = tuple(int(g.integers(lo, top + 1)) for _ in range(d))
        lam = float(g.uniform(2.0, 20.0))
        out.append((dims, lam))
    return out
