"""Helpers for the GPU parity tests: stored inputs built on the host (never by
the HIP path) and exact host views of what the device holds."""
import numpy as np
import torch

from oracle import quant as Q
from paper_2501_03121_amd import synth

TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-5, "bf16": 1e-5, "e4m3": 1e-5}
TORCH = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16,
         "e4m3": torch.float8_e4m3fn}


def stored_tensor(dims, fmt, seed, dev, kind="uniform"):
    """(device tensor, device scales or None, exact float64 host values).

    f16/bf16 values are cast on the host by torch's CPU conversion; E4M3
    tensors are random finite codes with random per-slice scales."""
    dims = tuple(int(n) for n in dims)
    if fmt == "e4m3":
        g = synth.rng(seed)
        codes = g.integers(0, 256, size=dims).astype(np.uint8)
        codes[(codes & 0x7F) == 0x7F] = 0x7E
        scale = g.uniform(0.01, 2.0, size=dims[0]).astype(np.float32)
        A = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(dev)
        S = torch.from_numpy(scale).to(dev)
        return A, S, Q.dequantize_e4m3_slabs(codes, scale)
    base = synth.uniform(dims, seed) if kind == "uniform" else synth.normal(dims, seed)
    if fmt == "f64":
        host = torch.from_numpy(base)
    else:
        host = torch.from_numpy(base.astype(np.float32)).to(TORCH[fmt])
    exact = host.to(torch.float64).numpy()
    return host.to(dev), None, exact


def vec(n, seed, fmt, dev):
    x = synth.uniform(n, seed)
    x = x / np.linalg.norm(x)
    dt = torch.float64 if fmt == "f64" else torch.float32
    xt = torch.from_numpy(x).to(dt)
    return xt.to(dev), xt.to(torch.float64).numpy()


def host(t):
    return t.detach().cpu().to(torch.float64).numpy()


# unit roundoff of the accumulation type (float64 data accumulate in double,
# every other format in float)
UNIT = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "f16": 2.0 ** -24, "bf16": 2.0 ** -24,
        "e4m3": 2.0 ** -24}


def assert_elementwise(got, ref, ref_abs, n, fmt, what=""):
    """Every output within the rounding bound of an n-term dot product in the
    accumulation type: |got - ref| <= (2n + 8) u sum |a_i x_i| (ref_abs is
    that sum of magnitudes, from the oracle on |A| and |x|).  Any summation
    order meets it, so a single wrong output cannot hide under a norm."""
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    ref_abs = np.asarray(ref_abs, dtype=np.float64).reshape(-1)
    bound = (2 * n + 8) * UNIT[fmt] * ref_abs + 1e-300
    bad = np.flatnonzero(np.abs(got - ref) > bound)
    assert bad.size == 0, (what, fmt, int(bad.size), int(bad[0]), float(got[bad[0]]),
                           float(ref[bad[0]]), float(bound[bad[0]]))
