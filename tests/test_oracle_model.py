"""Pins for the oracle's forward pass: brute force, textbook convolution, causality,
receptive field, linearity, closed forms, window/stream equivalence."""
import numpy as np
import pytest

from oracle.arch import FULL, TINY, Arch, layout, num_params, pack, receptive_field, unpack
from oracle.forward import causal_conv, forward_stream, forward_window, gated_layer, sigmoid
from oracle.stream import ensemble, gather_windows, n_windows, owner, stitch
from paper_2201_11133_amd import synth

SMALL1 = Arch(kind=1, in_channels=2, channels=3, skip_channels=4, head_channels=3,
              n_stacks=2, layers_per_stack=3, kernel_size=2, input_kernel=1, head_mid_relu=0)
SMALL1_MID = Arch(**{**SMALL1.__dict__, "head_mid_relu": 1})
SMALL0 = Arch(kind=0, in_channels=2, channels=3, skip_channels=0, head_channels=0,
              n_stacks=1, layers_per_stack=3, kernel_size=2)


def rand_blob(a, seed, scale=0.7):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(num_params(a)) * scale


def test_param_counts_and_rf():
    assert num_params(TINY) == 1681
    assert num_params(FULL) == 2964993
    assert receptive_field(TINY) == 16
    assert receptive_field(FULL) == 3070
    assert receptive_field(Arch(input_kernel=2)) == 3071
    # keeping the dead last residual would give 2,981,505
    assert num_params(FULL) + 128 * 128 + 128 == 2981505


def test_generator_layout_matches_oracle_layout():
    for a, kw in [(TINY, synth.TINY_LAYOUT), (FULL, synth.FULL_LAYOUT)]:
        ours = [(s, f) for _, s, f in layout(a)]
        assert ours == synth.weight_layout(**kw)


def test_pack_unpack_roundtrip():
    b = rand_blob(FULL, 3)
    assert np.array_equal(pack(FULL, unpack(FULL, b)), b)


# ---------------------------------------------------------------- brute force
def brute_conv(x, W, b, d):
    T, cin = x.shape
    cout, _, k = W.shape
    y = [[0.0] * cout for _ in range(T)]
    for t in range(T):
        for o in range(cout):
            s = float(b[o])
            for j in range(k):
                tau = t - (k - 1 - j) * d
                if tau < 0:
                    continue
                for c in range(cin):
                    s += float(W[o, c, j]) * float(x[tau, c])
            y[t][o] = s
    return np.array(y)


def brute_forward(a, p, u):
    """Pure-Python loops for the whole network on one window u [T, 2]."""
    import math
    T = u.shape[0]
    if a.kind == 0:
        y = u
        for i in range(a.n_layers):
            y = np.maximum(brute_conv(y, p[f"conv{i}.W"], p[f"conv{i}.b"], a.dilation(i)), 0.0)
        return np.array([sum(p["out.W"][0, c] * y[t, c] for c in range(a.channels)) + p["out.b"][0] for t in range(T)])
    C = a.channels
    x = np.array([[sum(p["in.W"][o, c] * u[t, c] for c in range(2)) + p["in.b"][o] for o in range(C)] for t in range(T)])
    skip = np.zeros((T, a.skip_channels))
    for l in range(a.n_layers):
        pre = brute_conv(x, p[f"dil{l}.W"], p[f"dil{l}.b"], a.dilation(l))
        g = np.array([[math.tanh(pre[t, c]) / (1.0 + math.exp(-pre[t, C + c])) for c in range(C)] for t in range(T)])
        for t in range(T):
            for o in range(a.skip_channels):
                skip[t, o] += sum(p[f"skip{l}.W"][o, c] * g[t, c] for c in range(C)) + p[f"skip{l}.b"][o]
        if l < a.n_layers - 1:
            xn = x.copy()
            for t in range(T):
                for o in range(C):
                    xn[t, o] += sum(p[f"res{l}.W"][o, c] * g[t, c] for c in range(C)) + p[f"res{l}.b"][o]
            x = xn
    z = []
    for t in range(T):
        r = [max(v, 0.0) for v in skip[t]]
        h = [sum(p["h1.W"][o, c] * r[c] for c in range(a.skip_channels)) + p["h1.b"][o] for o in range(a.head_channels)]
        if a.head_mid_relu:
            h = [max(v, 0.0) for v in h]
        z.append(sum(p["h2.W"][0, c] * h[c] for c in range(a.head_channels)) + p["h2.b"][0])
    return np.array(z)


@pytest.mark.parametrize("d", [1, 2, 5, 64])
def test_causal_conv_vs_brute(d):
    rng = np.random.default_rng(d)
    x = rng.standard_normal((40, 3))
    W = rng.standard_normal((4, 3, 2))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(causal_conv(x, W, b, d), brute_conv(x, W, b, d), rtol=0, atol=1e-12)


def test_causal_conv_vs_numpy_convolve():
    """Textbook: output channel o = b_o + sum_c conv(x_c, [w1, 0 ... 0, w0]) (dilated kernel, full mode, truncated)."""
    rng = np.random.default_rng(11)
    T, cin, cout, d = 50, 3, 2, 4
    x = rng.standard_normal((T, cin))
    W = rng.standard_normal((cout, cin, 2))
    b = rng.standard_normal(cout)
    ref = np.zeros((T, cout))
    for o in range(cout):
        ref[:, o] = b[o]
        for c in range(cin):
            ker = np.zeros(d + 1)
            ker[0] = W[o, c, 1]      # current sample
            ker[d] = W[o, c, 0]      # sample d steps back
            ref[:, o] += np.convolve(x[:, c], ker, mode="full")[:T]
    np.testing.assert_allclose(causal_conv(x, W, b, d), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("a", [SMALL0, SMALL1, SMALL1_MID], ids=["kind0", "kind1", "kind1_midrelu"])
def test_forward_vs_brute(a):
    rng = np.random.default_rng(5)
    p = unpack(a, rand_blob(a, 7))
    u = rng.standard_normal((48, 2))
    np.testing.assert_allclose(forward_window(a, p, u), brute_forward(a, p, u), rtol=0, atol=1e-10)


def test_tiny_member_vs_brute():
    rng = np.random.default_rng(6)
    p = unpack(TINY, synth.tiny_weights(0).astype(np.float64))
    u = rng.standard_normal((40, 2))
    np.testing.assert_allclose(forward_window(TINY, p, u), brute_forward(TINY, p, u), rtol=0, atol=1e-10)


# ---------------------------------------------------------------- causality and receptive field
@pytest.mark.parametrize("a", [TINY, SMALL1], ids=["tiny", "small1"])
def test_causality(a):
    rng = np.random.default_rng(1)
    p = unpack(a, rand_blob(a, 2))
    u = rng.standard_normal((128, 2))
    z = forward_window(a, p, u)
    for t in [0, 17, 90]:
        v = u.copy()
        v[t + 1:] += rng.standard_normal(v[t + 1:].shape) * 5
        z2 = forward_window(a, p, v)
        assert np.array_equal(z[:t + 1], z2[:t + 1])
        assert not np.array_equal(z[t + 1:], z2[t + 1:])


@pytest.mark.parametrize("a", [TINY, SMALL1, FULL], ids=["tiny", "small1", "full"])
def test_receptive_field(a):
    rng = np.random.default_rng(4)
    p = unpack(a, synth.tiny_weights(0).astype(np.float64) if a is TINY else
               (synth.full_weights(1).astype(np.float64) if a is FULL else rand_blob(a, 3)))
    rf = receptive_field(a)
    T = rf + 8
    u = rng.standard_normal((T, 2))
    t = T - 1
    z = forward_window(a, p, u)
    v = u.copy()
    v[t - rf] += 3.0                  # outside the field: no effect on z[t]
    assert forward_window(a, p, v)[t] == z[t]
    v = u.copy()
    v[t - rf + 1] += 3.0              # oldest sample inside the field
    assert forward_window(a, p, v)[t] != z[t]


# ---------------------------------------------------------------- linearity of the pre-activation
def test_preactivation_linear_in_input_and_weights():
    rng = np.random.default_rng(9)
    a = SMALL1
    p = unpack(a, rand_blob(a, 4))
    x1, x2 = rng.standard_normal((2, 30, a.channels))
    skip = np.zeros((30, a.skip_channels))
    al, be = 0.37, -1.9
    pz = dict(p)
    pz["dil1.b"] = np.zeros_like(p["dil1.b"])
    pre = lambda q, x: gated_layer(a, q, 1, x, skip)[0]
    np.testing.assert_allclose(pre(pz, al * x1 + be * x2), al * pre(pz, x1) + be * pre(pz, x2), atol=1e-12)
    q1, q2, q3 = dict(pz), dict(pz), dict(pz)
    Wa, Wb = rng.standard_normal((2,) + p["dil1.W"].shape)
    q1["dil1.W"], q2["dil1.W"], q3["dil1.W"] = Wa, Wb, al * Wa + be * Wb
    np.testing.assert_allclose(pre(q3, x1), al * pre(q1, x1) + be * pre(q2, x1), atol=1e-12)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("mid", [0, 1])
def test_closed_form_zero_dilated_weights(mid):
    """dil.W = 0 and filter biases 0 => g = 0 => z = w_h2 . act(W_h1 ReLU(sum_l b_s^l) + b_h1) + b_h2 everywhere."""
    a = Arch(**{**FULL.__dict__, "head_mid_relu": mid})
    rng = np.random.default_rng(12)
    p = unpack(a, rng.standard_normal(num_params(a)))
    for l in range(a.n_layers):
        p[f"dil{l}.W"][:] = 0
        p[f"dil{l}.b"][:a.channels] = 0
    u = rng.standard_normal((64, 2))
    z = forward_window(a, p, u)
    sb = sum(p[f"skip{l}.b"] for l in range(a.n_layers))
    h = p["h1.W"] @ np.maximum(sb, 0) + p["h1.b"]
    if mid:
        h = np.maximum(h, 0)
    zc = float(p["h2.W"][0] @ h + p["h2.b"][0])
    np.testing.assert_allclose(z, zc, rtol=1e-12, atol=1e-12)


def test_closed_form_tiny_zero_conv():
    rng = np.random.default_rng(13)
    p = unpack(TINY, rng.standard_normal(num_params(TINY)))
    for i in range(4):
        p[f"conv{i}.W"][:] = 0
    z = forward_window(TINY, p, rng.standard_normal((32, 2)))
    np.testing.assert_allclose(z, p["out.W"][0] @ np.maximum(p["conv3.b"], 0) + p["out.b"][0], atol=1e-12)


# ---------------------------------------------------------------- windows, stitching, ensemble
def test_window_count_and_owner():
    W, S = 4096, 256
    assert n_windows(0, W, S) == 0
    assert n_windows(10, W, S) == 1
    assert n_windows(W, W, S) == 1
    assert n_windows(W + 1, W, S) == 2
    assert n_windows(16777216, W, S) == 65521
    assert n_windows(353894400, W, S) == 1382385
    k, pos = owner(np.array([0, W - S - 1, W - S, W - 1, W, W + S - 1, W + S]), W, S)
    assert list(k) == [0, 0, 0, 0, 1, 1, 2]
    assert list(pos) == [0, W - S - 1, W - S, W - 1, W - S, W - 1, W - S]
    # every owner position is inside its window and every window after the first owns exactly S samples
    L = 20000
    k, pos = owner(np.arange(L), W, S)
    assert k.max() == n_windows(L, W, S) - 1 and pos.min() >= 0 and pos.max() < W
    assert np.all(pos[L // 2:] >= W - S)


def test_window_vs_stream_equivalence():
    """Owner-window stitched scores equal a single causal pass over the stream (RF - 1 <= W - S)."""
    a = SMALL1
    rng = np.random.default_rng(21)
    p = unpack(a, rand_blob(a, 5))
    W, S = 32, 8
    assert receptive_field(a) - 1 <= W - S
    for L in [5, 32, 33, 100, 123]:
        u = rng.standard_normal((L, 2))
        zw = forward_window(a, p, gather_windows(u, W, S))
        np.testing.assert_allclose(stitch(zw, L, W, S), forward_stream(a, p, u), rtol=0, atol=1e-12)


def test_window_vs_stream_tiny_member_real_shape():
    rng = np.random.default_rng(22)
    p = unpack(TINY, synth.tiny_weights(0).astype(np.float64))
    W, S, L = 4096, 256, 4096 + 3 * 256 + 77
    u = rng.standard_normal((L, 2))
    zw = forward_window(TINY, p, gather_windows(u, W, S))
    np.testing.assert_allclose(stitch(zw, L, W, S), forward_stream(TINY, p, u), rtol=0, atol=1e-12)


def test_ensemble_min():
    rng = np.random.default_rng(3)
    z = rng.standard_normal(100)
    assert np.array_equal(ensemble([z, z, z]), z)
    z2 = rng.standard_normal(100)
    e = ensemble([z, z2])
    assert np.array_equal(e, np.where(z < z2, z, z2))
    # agreement: e >= thr exactly when every member is
    thr = np.log(9.0)
    assert np.array_equal(e >= thr, (z >= thr) & (z2 >= thr))


def test_sigmoid_threshold_equivalence():
    z = np.linspace(-10, 10, 100001)
    assert np.array_equal(sigmoid(z) >= 0.9, z >= np.log(9.0)) or \
        np.count_nonzero((sigmoid(z) >= 0.9) != (z >= np.log(9.0))) <= 1
