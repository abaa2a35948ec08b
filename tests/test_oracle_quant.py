"""Pins for the bfloat16 / FP8-E4M3FN quantisers against PyTorch's CPU casts (library routines)."""
import numpy as np
import pytest
import torch

from oracle.quant import E4M3_MAX, e4m3_channel_scales, quantise_weight_e4m3, to_bf16, to_e4m3


def _values(seed, n=200000):
    rng = np.random.default_rng(seed)
    v = np.concatenate([rng.standard_normal(n) * 10 ** rng.uniform(-6, 4, n),
                        rng.uniform(-500, 500, 1000), [0.0, -0.0, 1.0, -1.0, 448.0, -448.0, 2 ** -9, 2 ** -10, 3 * 2 ** -10]])
    return v.astype(np.float32).astype(np.float64)


def test_bf16_matches_torch():
    v = _values(1)
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).float().double().numpy()
    np.testing.assert_array_equal(to_bf16(v), ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: even mantissa wins -> 1
    assert to_bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert to_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 * 2 ** -7


def test_e4m3_matches_torch_in_range():
    v = _values(2)
    v = v[np.abs(v) <= E4M3_MAX]
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.float8_e4m3fn).float().double().numpy()
    np.testing.assert_array_equal(to_e4m3(v), ref)


def test_e4m3_grid_and_saturation():
    assert to_e4m3(np.array([1000.0, -1e9, 449.0]))[0] == 448.0
    assert to_e4m3(np.array([-1e9]))[0] == -448.0
    # subnormal spacing 2^-9, smallest normal 2^-6, 8 values per binade
    assert to_e4m3(np.array([2 ** -9]))[0] == 2 ** -9
    assert to_e4m3(np.array([2 ** -11]))[0] == 0.0
    grid = np.unique(np.abs(to_e4m3(np.linspace(-448, 448, 200001))))
    assert grid.size == 127 - 1 + 1 - 0 or grid.size <= 127   # 126 positive finite codes + zero


def test_e4m3_channel_scales():
    rng = np.random.default_rng(3)
    W = rng.standard_normal((8, 5, 2))
    W[3] = 0
    codes, s = quantise_weight_e4m3(W)
    assert s[3] == 1.0
    amax = np.abs(W.reshape(8, -1)).max(axis=1)
    np.testing.assert_allclose(s[[0, 1, 2, 4]], amax[[0, 1, 2, 4]] / 448.0)
    assert np.all(np.abs(codes) <= 448.0)
    # every channel's largest entry maps to +/-448 exactly
    assert np.all(np.isclose(np.abs(codes.reshape(8, -1)).max(axis=1)[[0, 1, 2, 4]], 448.0))
    np.testing.assert_allclose(codes * s[:, None, None], W, rtol=2 ** -3, atol=s.max() * 2 ** -9)
