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


def _torch_weight_e4m3_f32(W):
    """Independent statement of the float32 per-output-channel quantiser, in torch float32 CPU
    arithmetic: s = fl32(max |w| / 448) (1 for an all-zero channel), code = e4m3fn(fl32(w / s))."""
    W32 = torch.from_numpy(np.ascontiguousarray(W, dtype=np.float32))
    amax = W32.abs().reshape(W32.shape[0], -1).amax(dim=1)
    s = torch.where(amax > 0, amax / torch.tensor(448.0, dtype=torch.float32), torch.ones_like(amax))
    q = W32 / s.reshape((-1,) + (1,) * (W32.dim() - 1))
    return q.to(torch.float8_e4m3fn).double().numpy(), s.numpy()


def test_quantise_weight_e4m3_f32_matches_torch():
    """The float32 form of the FP8 weight quantiser (the library exports its codes and scales and the
    GPU tests compare them bit for bit) against torch float32 division and the float8_e4m3fn cast:
    random channels over many magnitudes, all-zero channels, and channels built so that w / s lands
    exactly halfway between two E4M3 values (ties to even)."""
    from oracle.quant import quantise_weight_e4m3_f32
    rng = np.random.default_rng(7)
    n_out, n_in = 4096, 24
    W = rng.standard_normal((n_out, n_in, 2)) * 10.0 ** rng.uniform(-5, 3, (n_out, 1, 1))
    W[5] = 0.0
    W[77] = 0.0
    # amax = 448 * 2^k gives s = 2^k exactly; 1.0625 and 1.1875 are ties between E4M3 neighbours
    for i, k in zip(range(100, 110), range(-5, 5)):
        W[i] = 0.0
        W[i, 0, 0] = 448.0 * 2.0 ** k
        W[i, 1, 0] = 1.0625 * 2.0 ** k      # halfway 1 / 1.125: even mantissa -> 1
        W[i, 2, 1] = -1.1875 * 2.0 ** k     # halfway 1.125 / 1.25 -> -1.25
        W[i, 3, 1] = 3.0 * 2.0 ** (k - 10)  # subnormal range of the code grid
    codes, s = quantise_weight_e4m3_f32(W)
    ref_codes, ref_s = _torch_weight_e4m3_f32(W)
    assert s.dtype == np.float32
    np.testing.assert_array_equal(s, ref_s)
    np.testing.assert_array_equal(codes, ref_codes)
    assert s[5] == 1.0 and s[77] == 1.0 and not codes[5].any()
    for i, k in zip(range(100, 110), range(-5, 5)):
        assert s[i] == np.float32(2.0 ** k)
        assert codes[i, 0, 0] == 448.0 and codes[i, 1, 0] == 1.0 and codes[i, 2, 1] == -1.25
    # the pin has power: the scale taken as amax * fl32(1 / 448) differs on some channel
    amax = np.abs(W.astype(np.float32).reshape(n_out, -1)).max(axis=1)
    alt = (amax * np.float32(1.0 / 448.0)).astype(np.float32)
    assert np.any((alt != s) & (amax > 0))
