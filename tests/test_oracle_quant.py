"""Pins of the storage-format oracle: the OCP E4M3 format definition, exact
round trips, and library conversions (numpy / torch CPU) as independent
opinions.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import quant as Q
from paper_2501_03121_amd import synth


def test_e4m3_known_codes():
    vals = Q.e4m3_to_f64(np.array([0x00, 0x80, 0x01, 0x07, 0x08, 0x38, 0xB8, 0x7E, 0xFE, 0x7F, 0xFF, 0x40],
                                  dtype=np.uint8))
    assert vals[0] == 0.0 and np.signbit(vals[1])
    assert vals[2] == 2.0 ** -9 and vals[3] == 7 * 2.0 ** -9 and vals[4] == 2.0 ** -6
    assert vals[5] == 1.0 and vals[6] == -1.0
    assert vals[7] == 448.0 and vals[8] == -448.0
    assert np.isnan(vals[9]) and np.isnan(vals[10])
    assert vals[11] == 2.0


def test_e4m3_decode_matches_torch():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = Q.e4m3_to_f64(codes)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(got[ok], ref[ok])


def test_e4m3_round_trip_all_codes():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    vals = Q.e4m3_to_f64(codes).astype(np.float32)
    assert np.array_equal(Q.e4m3_from_f32(vals), codes)


def test_e4m3_encode_matches_torch_rne():
    # random values plus every midpoint between neighbouring codes (ties to even)
    r = synth.normal(20000, 5, std=30.0).astype(np.float32)
    r = r[np.abs(r) < 460]
    pos = Q.e4m3_to_f64(np.arange(0, 0x7F, dtype=np.uint8))
    mids = ((pos[:-1] + pos[1:]) / 2).astype(np.float32)
    vals = np.concatenate([r, mids, -mids, np.float32([0.0, 1e-9, -1e-9, 447.9, 300.5])])
    ref = torch.from_numpy(vals).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = Q.e4m3_from_f32(vals)
    # torch keeps the sign of values that round to zero; so do we
    assert np.array_equal(got, ref)


def test_e4m3_saturation_and_nan():
    v = np.float32([1000.0, -1000.0, np.inf, -np.inf, np.nan, 449.0])
    assert list(Q.e4m3_from_f32(v)) == [0x7E, 0xFE, 0x7E, 0xFE, 0x7F, 0x7E]


def test_bf16_rne_and_truncation():
    v = np.concatenate([synth.normal(5000, 6, std=100).astype(np.float32),
                        np.float32([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 3.0e38, 0.0])])
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(Q.bf16_from_f32_rne(v), ref)
    assert np.array_equal(Q.bf16_from_f32_trunc(v), (v.view(np.uint32) >> 16).astype(np.uint16))
    back = Q.bf16_to_f64(Q.bf16_from_f32_rne(v))
    assert np.all(np.abs(back - v) <= 2.0 ** -8 * np.abs(v))


def test_f16_matches_torch():
    v = synth.normal(5000, 7, std=50).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.float16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(Q.f16_from_f32(v), ref)
    assert np.array_equal(Q.f16_to_f64(ref), torch.from_numpy(v).half().double().numpy())


def test_slab_scales_and_error_bound():
    A = synth.normal((6, 7, 5), 8).astype(np.float32)
    A[2] = 0.0
    codes, s = Q.quantize_e4m3_slabs(A)
    assert s[2] == 1.0 and np.all(codes[2] == 0)
    for i in range(6):
        if i == 2:
            continue
        assert s[i] == np.float32(np.abs(A[i]).max() / np.float32(448.0))
        assert np.max(codes[i] & 0x7F) == 0x7E   # the absmax lands on +-448
    deq = Q.dequantize_e4m3_slabs(codes, s)
    bound = 2.0 ** -4 * np.abs(A) + s.reshape(6, 1, 1) * 2.0 ** -10
    assert np.all(np.abs(deq - A) <= bound * (1 + 1e-6))
