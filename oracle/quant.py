"""Oracle for the low-precision storage formats (test infrastructure only).

The paper stores tensors in a low-precision format and promotes every value to
the higher precision before any arithmetic (Sec. 5.5): IEEE binary16 ("half"),
and "brain" 16-bit floats made by truncating binary32.  OCP FP8 E4M3 (FN
variant) with one float32 scale per mode-0 slice is a further format of this
library, not of the paper.

Readings:
  * bf16 is produced with round-to-nearest-even by default; truncation (the
    paper's conversion) is available as `bf16_from_f32_trunc`.
  * E4M3 (OCP, "FN"): 1 sign bit, 4 exponent bits with bias 7, 3 mantissa bits,
    no infinities, NaN only at S.1111.111, largest finite value 448, smallest
    subnormal 2^-9.  Encoding rounds to nearest even and saturates finite
    values beyond 448 to +-448.
  * Slab scale s_i = absmax(A[i, ...]) / 448 computed in float32 (s_i = 1 for
    an all-zero slab); codes are e4m3(float32(A / s_i)) with the division done
    in float32; the value a code stands for is decode(code) * s_i.

The oracle decodes stored bits exactly (into float64).
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


# ---------------------------------------------------------------- bf16
def bf16_from_f32_rne(a: np.ndarray) -> np.ndarray:
    """float32 -> bf16 bit patterns (uint16), round to nearest, ties to even."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16).astype(np.uint32)
    nan = np.isnan(a)
    if nan.any():
        sign = (bits >> 31).astype(np.uint32)
        rounded = np.where(nan, (sign << 15) | 0x7FC0, rounded)
    return rounded.astype(np.uint16)


def bf16_from_f32_trunc(a: np.ndarray) -> np.ndarray:
    """float32 -> bf16 bit patterns by dropping the low 16 bits (truncation)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    return (a.view(np.uint32) >> 16).astype(np.uint16)


def bf16_to_f64(u: np.ndarray) -> np.ndarray:
    """bf16 bit patterns -> exact float64 values."""
    u = np.asarray(u, dtype=np.uint16)
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- fp16
def f16_from_f32(a: np.ndarray) -> np.ndarray:
    """float32 -> IEEE binary16 bit patterns, round to nearest even (library
    conversion)."""
    return np.asarray(a, dtype=np.float32).astype(np.float16).view(np.uint16)


def f16_to_f64(u: np.ndarray) -> np.ndarray:
    """binary16 bit patterns -> exact float64 values."""
    return np.asarray(u, dtype=np.uint16).view(np.float16).astype(np.float64)


# ---------------------------------------------------------------- e4m3
def e4m3_to_f64(c: np.ndarray) -> np.ndarray:
    """E4M3 codes (uint8) -> exact float64 values (NaN for S.1111.111)."""
    c = np.asarray(c, dtype=np.uint8).astype(np.int64)
    sign = np.where(c >> 7, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    normal = (1.0 + m / 8.0) * np.exp2(e - 7.0)
    sub = m * 2.0 ** -9
    val = np.where(e == 0, sub, normal)
    val = np.where((e == 15) & (m == 7), np.nan, val)
    return sign * val


def e4m3_from_f32(a: np.ndarray) -> np.ndarray:
    """float32 -> E4M3 codes: round to nearest even, finite overflow saturates
    to +-448, NaN -> S.1111.111."""
    a32 = np.asarray(a, dtype=np.float32)
    v = a32.astype(np.float64)
    sign = np.signbit(a32).astype(np.uint8)
    mag = np.abs(v)
    out = np.zeros(v.shape, dtype=np.uint8)
    nan = np.isnan(mag)
    big = (~nan) & (mag >= E4M3_MAX)
    sub = (~nan) & (~big) & (mag < 2.0 ** -6)
    nrm = (~nan) & (~big) & (~sub)
    # subnormal range: multiples of 2^-9; q = 8 lands exactly on code 0x08 (2^-6)
    q_sub = np.rint(mag[sub] * 2.0 ** 9)           # rint = round half to even
    out[sub] = q_sub.astype(np.uint8)
    # normal range: value = (1 + q/8) 2^e
    mant, ex = np.frexp(mag[nrm])                  # mag = mant * 2^ex, mant in [0.5, 1)
    e = ex.astype(np.int64) - 1                    # mag = (2 mant) 2^e, 2 mant in [1, 2)
    q = np.rint((2.0 * mant - 1.0) * 8.0).astype(np.int64)
    carry = q == 8
    e = np.where(carry, e + 1, e)
    q = np.where(carry, 0, q)
    out[nrm] = (((e + 7) << 3) | q).astype(np.uint8)
    out[big] = 0x7E
    out[nan] = 0x7F
    return out | (sign << 7)


def slab_scales(A: np.ndarray) -> np.ndarray:
    """Per mode-0 slice scale absmax / 448 in float32 (1 for an all-zero slice)."""
    A32 = np.asarray(A, dtype=np.float32)
    amax = np.abs(A32.reshape(A32.shape[0], -1)).max(axis=1).astype(np.float32)
    s = (amax / np.float32(E4M3_MAX)).astype(np.float32)
    return np.where(amax == 0, np.float32(1.0), s).astype(np.float32)


def quantize_e4m3_slabs(A: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(codes, scales): codes = e4m3(float32(A / s_i)) per mode-0 slice i."""
    A32 = np.asarray(A, dtype=np.float32)
    s = slab_scales(A32)
    shp = (A32.shape[0],) + (1,) * (A32.ndim - 1)
    q = (A32 / s.reshape(shp)).astype(np.float32)
    return e4m3_from_f32(q), s


def dequantize_e4m3_slabs(codes: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """Exact float64 values the stored codes and scales stand for."""
    c = np.asarray(codes, dtype=np.uint8)
    shp = (c.shape[0],) + (1,) * (c.ndim - 1)
    return e4m3_to_f64(c) * np.asarray(scales, dtype=np.float64).reshape(shp)
