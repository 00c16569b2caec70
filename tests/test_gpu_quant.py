"""The HIP storage conversions (tvc_quantize) against the bit-level oracle,
and the hardware E4M3 decode the contraction kernels use."""
import numpy as np
import pytest
import torch

import paper_2501_03121_amd as tvc
from oracle import quant as Q
from paper_2501_03121_amd import synth

pytestmark = pytest.mark.gpu


def as_bits(t):
    return t.cpu().view(torch.uint8 if t.element_size() == 1 else torch.int16).numpy().view(
        np.uint8 if t.element_size() == 1 else np.uint16)


@pytest.mark.parametrize("dims", [(64, 33, 17), (1000,), (3, 70000)])
def test_bf16_f16_bits(dev, dims):
    v = synth.normal(dims, 1, std=20).astype(np.float32)
    v.reshape(-1)[:4] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 0.0, -2.5]
    A = torch.from_numpy(v).to(dev)
    b, _ = tvc.quantize(A, "bf16")
    assert np.array_equal(as_bits(b), Q.bf16_from_f32_rne(v))
    t, _ = tvc.quantize(A, "bf16", truncate=True)
    assert np.array_equal(as_bits(t), Q.bf16_from_f32_trunc(v))
    h, _ = tvc.quantize(A, "f16")
    assert np.array_equal(as_bits(h), Q.f16_from_f32(v))


@pytest.mark.parametrize("dims", [(16, 40, 30), (5, 300000), (7, 1)])
def test_e4m3_codes_and_scales(dev, dims):
    v = synth.normal(dims, 2, std=3).astype(np.float32)
    v[-1] = 0.0
    A = torch.from_numpy(v).to(dev)
    q, s = tvc.quantize(A, "e4m3")
    codes, scales = Q.quantize_e4m3_slabs(v)
    assert np.array_equal(s.cpu().numpy(), scales)
    assert np.array_equal(as_bits(q), codes)


def test_hardware_e4m3_decode_table(dev):
    # every finite code through the contraction kernel: one-hot weights read
    # each element back as decode(code) * scale
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    n = codes.shape[0]
    A = torch.from_numpy(codes.reshape(n, 1)).view(torch.float8_e4m3fn).to(dev)
    S = torch.ones(n, dtype=torch.float32, device=dev)
    y = tvc.contract(A, torch.ones(1, dtype=torch.float32, device=dev), 1, scale=S)
    assert np.array_equal(y.cpu().double().numpy(), Q.e4m3_to_f64(codes))
