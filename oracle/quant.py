"""Reduced-precision formats written from their definitions (oracle).

Test infrastructure only (see the package docstring).

The paper lets its inference engine use half precision where possible
("Optimization with TensorRT"). The build's reduced-precision forms are
bfloat16 and FP8 E4M3 (OCP "FN" variant: 4 exponent bits with bias 7, 3
mantissa bits, no infinities, largest finite value 448). Both quantisers
round to nearest, ties to even. Reading: FP8 values beyond +/-448 saturate to
+/-448; weights get one scale per output channel, amax over that channel's
entries (both taps) / 448; activations use a unit scale.
"""
from __future__ import annotations

import numpy as np


def _round_to_grid(x: np.ndarray, man_bits: int, min_exp: int) -> np.ndarray:
    """Round finite x to the nearest value with `man_bits` fraction bits, ties to even.

    Normal numbers |x| in [2^e, 2^(e+1)) have spacing 2^(e - man_bits); below
    2^min_exp the spacing stays 2^(min_exp - man_bits) (subnormals).
    """
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    _, E = np.frexp(ax)                     # ax = m 2^E, m in [0.5, 1)
    e = np.maximum(E - 1, min_exp)
    q = np.ldexp(1.0, e - man_bits)
    return np.sign(x) * np.rint(ax / q) * q


def to_bf16(x: np.ndarray) -> np.ndarray:
    """float64 -> nearest bfloat16 value (8 exponent bits, 7 fraction bits), returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    r = _round_to_grid(x, 7, -126)
    max_bf16 = (2.0 - 2.0 ** -7) * 2.0 ** 127
    # a value at or past max + half a spacing overflows to infinity under round-to-nearest
    over = np.abs(x) >= max_bf16 + 2.0 ** (127 - 8)
    return np.where(over, np.copysign(np.inf, x), r)


E4M3_MAX = 448.0


def to_e4m3(x: np.ndarray) -> np.ndarray:
    """float64 -> nearest FP8 E4M3FN value (bias 7, 3 fraction bits), saturating at +/-448."""
    r = _round_to_grid(x, 3, -6)
    return np.clip(r, -E4M3_MAX, E4M3_MAX)


def e4m3_channel_scales(W: np.ndarray) -> np.ndarray:
    """Per-output-channel scale (axis 0) = max |W| over the channel / 448 (1 for an all-zero channel)."""
    W = np.asarray(W, dtype=np.float64)
    amax = np.max(np.abs(W.reshape(W.shape[0], -1)), axis=1)
    return np.where(amax > 0, amax / E4M3_MAX, 1.0)


def quantise_weight_e4m3_f32(W: np.ndarray):
    """Same quantiser with the scale and the division taken in float32 (as a float32 kernel does):
    s = float32(max |w|) / 448, code = e4m3(float32(w) / s). Returns (codes, scales as float32)."""
    W32 = np.asarray(W, dtype=np.float32)
    amax = np.max(np.abs(W32.reshape(W32.shape[0], -1)), axis=1)
    s = np.where(amax > 0, amax / np.float32(E4M3_MAX), np.float32(1.0)).astype(np.float32)
    shape = (W32.shape[0],) + (1,) * (W32.ndim - 1)
    return to_e4m3((W32 / s.reshape(shape)).astype(np.float32).astype(np.float64)), s


def quantise_weight_e4m3(W: np.ndarray):
    """(codes as float64 values, scales): W ~= codes * scale[:, None, ...]."""
    W = np.asarray(W, dtype=np.float64)
    s = e4m3_channel_scales(W)
    shape = (W.shape[0],) + (1,) * (W.ndim - 1)
    return to_e4m3(W / s.reshape(shape)), s
