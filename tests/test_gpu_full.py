"""Parity at the benchmark's full sizes and launch configuration: 1024^3 and
32^6 float32 tensors (4.3 GB each) and their bf16, fp16 and E4M3 stored copies.  Contractions are checked on sampled
outputs that the oracle computes one by one from the exact host copy of the
device bytes; HOPM sweeps against the float64 canonical oracle from the same
start vectors."""
import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import hopm as H
from oracle import quant as Q
from oracle import tvc as O
from paper_2501_03121_amd import synth
from _util import host

pytestmark = pytest.mark.gpu

SHAPES = [(1024, 1024, 1024), (32, 32, 32, 32, 32, 32)]
SAMPLES = 2048


def sample_lr(dims, k, seed):
    u, _, v = O.matricized_dims(dims, k)
    g = synth.rng(seed)
    return np.stack([g.integers(0, u, SAMPLES), g.integers(0, v, SAMPLES)], axis=1)


@pytest.mark.parametrize("dims", SHAPES, ids=["1024^3", "32^6"])
def test_full_size_tvc_sampled(dev, dims):
    A = synth.device_normal(dims, 100, dev)
    Ah = A.cpu().numpy()
    Ab, _ = tvc.quantize(A, "bf16")
    Abh = Q.bf16_to_f64(Ab.cpu().view(torch.int16).numpy().view(np.uint16))
    for k in range(len(dims)):
        xh = synth.unit_vectors([dims[k]], 300 + k)[0].astype(np.float32)
        x = torch.from_numpy(xh).to(dev)
        lr = sample_lr(dims, k, 7 + k)
        u, _, v = O.matricized_dims(dims, k)
        y = host(tvc.contract(A, x, k)).reshape(u, v)[lr[:, 0], lr[:, 1]]
        ref = O.tvc_sample(Ah, xh, k, lr)
        assert O.rel_err(y, ref) < 1e-5, ("f32", dims, k, O.rel_err(y, ref))
        yb = host(tvc.contract(Ab, x, k)).reshape(u, v)[lr[:, 0], lr[:, 1]]
        refb = O.tvc_sample(Abh, xh, k, lr)
        assert O.rel_err(yb, refb) < 1e-5, ("bf16", dims, k)


class _Stored:
    """A stored tensor's codes; indexing a fiber [l, :, r] of its (u, n, v)
    view decodes that fiber alone to the exact values the codes stand for
    (the oracle's decoders; E4M3 codes times their mode-0 slab scale), so
    that the oracle can sample a full-size tensor without decoding it all."""

    def __init__(self, codes, decode, scale=None, view=None):
        self.codes, self.decode, self.scale = codes, decode, scale
        self.shape = codes.shape if view is None else view

    def reshape(self, u, n, v):
        return _Stored(self.codes, self.decode, self.scale, (u, n, v))

    def __getitem__(self, idx):
        l, _, r = idx
        _, n, v = self.shape
        flat = (l * n + np.arange(n, dtype=np.int64)) * v + r
        vals = self.decode(self.codes.reshape(-1)[flat])
        if self.scale is not None:
            slab = self.codes.size // self.codes.shape[0]
            vals = vals * self.scale.astype(np.float64)[flat // slab]
        return vals


@pytest.mark.parametrize("fmt", ["f16", "e4m3"])
@pytest.mark.parametrize("dims", SHAPES, ids=["1024^3", "32^6"])
def test_full_size_narrow_stored_values(dev, dims, fmt):
    # stored-value parity of fp16 and E4M3 (slab scales included) at full
    # size, every mode, on sampled outputs, each within 1e-5 of the
    # magnitude sum of its own terms
    A = synth.device_normal(dims, 100, dev)
    Aq, S = tvc.quantize(A, fmt)
    del A
    torch.cuda.empty_cache()
    if fmt == "f16":
        codes, dec = Aq.cpu().view(torch.int16).numpy().view(np.uint16), Q.f16_to_f64
    else:
        codes, dec = Aq.cpu().view(torch.uint8).numpy(), Q.e4m3_to_f64
    scale = None if S is None else S.cpu().numpy()
    exact = _Stored(codes, dec, scale)
    mag = _Stored(codes, lambda c: np.abs(dec(c)), scale)
    for k in range(len(dims)):
        xh = synth.unit_vectors([dims[k]], 300 + k)[0].astype(np.float32)
        x = torch.from_numpy(xh).to(dev)
        lr = sample_lr(dims, k, 7 + k)
        u, _, v = O.matricized_dims(dims, k)
        y = host(tvc.contract(Aq, x, k, scale=S)).reshape(u, v)[lr[:, 0], lr[:, 1]]
        ref = O.tvc_sample(exact, xh, k, lr)
        bound = O.tvc_sample(mag, np.abs(xh), k, lr)
        assert O.rel_err(y, ref) < 1e-5, (fmt, dims, k, O.rel_err(y, ref))
        worst = np.max(np.abs(y - ref) / bound)
        assert worst <= 1e-5, (fmt, dims, k, worst)


@pytest.mark.parametrize("dims", SHAPES, ids=["1024^3", "32^6"])
def test_full_size_hopm_sweep(dev, dims):
    A, a = synth.device_planted(dims, 10.0, 0.1, 200, dev)
    x0 = synth.warm_start(a, 0.9, 400)
    x = tvc.pack_vectors(x0, dev)
    r = tvc.read_stats(tvc.hopm_iterate(A, x, 1))
    ref = H.hopm(A.cpu().numpy(), x0, sweeps=1)
    got = np.split(host(x), np.cumsum(dims)[:-1])
    for g, e in zip(got, ref.xs):
        assert np.linalg.norm(g - e) < 1e-5
    assert abs(r.lam - ref.lam) < 1e-5 * ref.lam


@pytest.mark.timeout(600)
def test_full_size_bf16_lambda_error(dev):
    # 32^6 planted tensor: float64 oracle solve from the warm start vs the
    # bf16-storage solve, then float32 refinement sweeps to the same tol
    dims = SHAPES[1]
    A, a = synth.device_planted(dims, 10.0, 0.1, 200, dev)
    x0 = synth.warm_start(a, 0.9, 400)
    ref = H.hopm(A.cpu().numpy(), x0, tol=1e-6, max_sweeps=40)
    Ab, _ = tvc.quantize(A, "bf16")
    x = tvc.pack_vectors(x0, dev)
    r = tvc.hopm_solve(Ab, x, tol=1e-6, max_sweeps=200)
    assert r.status == 0 and r.delta < 1e-6
    assert abs(r.lam - ref.lam) <= 1e-3 * ref.lam
    r = tvc.hopm_solve(Ab, x, tol=1e-6, max_sweeps=200, A_refine=A, refine_sweeps=60)
    assert r.status == 0 and r.delta < 1e-6 and r.refine_sweeps >= 1
    assert abs(r.lam - ref.lam) <= 1e-5 * ref.lam
    x = tvc.pack_vectors(x0, dev)
    r32 = tvc.hopm_solve(A, x, tol=1e-6, max_sweeps=200)
    assert abs(r32.lam - ref.lam) <= 1e-5 * ref.lam


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dims", [(65537, 65537), (3, 65537, 21847)], ids=["65537^2", "3x65537x21847"])
def test_over_2e32_elements(dev, dims):
    # More than 2^32 elements (17.2 GB in float32) in every mode: 64-bit
    # element offsets, rows of more than 2^31 bytes cut into chunks, and the
    # 64-bit branch of the task index split.  Sampled outputs against the
    # oracle on the gathered fibers A[l, :, r].
    assert int(np.prod(dims)) > 2 ** 32
    A = synth.device_normal(dims, 120, dev)
    for k in range(len(dims)):
        xh = synth.unit_vectors([dims[k]], 320 + k)[0].astype(np.float32)
        y = tvc.contract(A, torch.from_numpy(xh).to(dev), k)
        u, n, v = O.matricized_dims(dims, k)
        g = synth.rng(11 + k)
        li = torch.from_numpy(g.integers(0, u, 64)).to(dev)
        ri = torch.from_numpy(g.integers(0, v, 64)).to(dev)
        fibers = host(A.view(u, n, v)[li, :, ri])            # (64, n), exact device values
        ref = O.tvc(fibers.reshape(64, n, 1), xh, 1).reshape(-1)
        got = host(y.view(u, v)[li, ri])
        assert O.rel_err(got, ref) < 1e-5, (dims, k)
        del y
    del A
    torch.cuda.empty_cache()
