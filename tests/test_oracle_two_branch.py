"""Pins for the two-branch member of the oracle (Fig. 1: one WaveNet branch per detector, the two
outputs concatenated, then two convolutions): parameter count in closed form, brute-force loops on a
tiny member, the block-diagonal identity with the single-trunk member, branch independence, and the
receptive field."""
import math

import numpy as np
import pytest

from oracle.arch import FULL, TWO_BRANCH, Arch, layout, num_params, pack, receptive_field, unpack
from oracle.forward import forward_window
from paper_2201_11133_amd import synth

TINY2 = Arch(kind=2, in_channels=2, channels=2, skip_channels=2, head_channels=3, n_stacks=1, layers_per_stack=3)


def rand_params(a, seed, scale=0.7):
    rng = np.random.default_rng(seed)
    return {n: rng.standard_normal(s) * scale for n, s, _ in layout(a)}


def test_param_count_closed_form():
    C, S, H, L = 64, 64, 128, 30
    branch = C * 1 + C + L * (2 * C * C * 2 + 2 * C) + (L - 1) * (C * C + C) + L * (S * C + S)
    assert num_params(TWO_BRANCH) == 2 * branch + H * 2 * S + H + H + 1 == 1_498_497
    assert receptive_field(TWO_BRANCH) == receptive_field(FULL) == 3070
    assert synth.two_branch_weights(3).size == num_params(TWO_BRANCH)
    # the generator's blob order is the oracle's: every weight tensor has the He-normal spread of its fan-in
    blob = synth.two_branch_weights(3).astype(np.float64)
    p = unpack(TWO_BRANCH, blob)
    for name, shape, fan in layout(TWO_BRANCH):
        if fan and np.prod(shape) >= 4096:
            assert abs(np.std(p[name]) / math.sqrt(2 / fan) - 1) < 0.1, name


def brute_two_branch(a, p, u):
    """Sample-by-sample loops: per-branch input projection, gated layers, skip sums; concatenation;
    head."""
    T = u.shape[0]
    C, S, H = a.channels, a.skip_channels, a.head_channels
    sig = lambda v: 1.0 / (1.0 + math.exp(-v))
    skips = []
    for br in range(2):
        q = lambda n: p[f"b{br}.{n}"]
        x = [[q("in.W")[c][0] * u[t][br] + q("in.b")[c] for c in range(C)] for t in range(T)]
        sk = [[0.0] * S for _ in range(T)]
        for l in range(a.n_layers):
            d = 2 ** (l % a.layers_per_stack)
            W, b = q(f"dil{l}.W"), q(f"dil{l}.b")
            xn = [row[:] for row in x]
            for t in range(T):
                pre = []
                for o in range(2 * C):
                    v = b[o]
                    for i in range(C):
                        v += W[o][i][1] * x[t][i] + (W[o][i][0] * x[t - d][i] if t - d >= 0 else 0.0)
                    pre.append(v)
                g = [math.tanh(pre[c]) * sig(pre[C + c]) for c in range(C)]
                for s_ in range(S):
                    sk[t][s_] += q(f"skip{l}.b")[s_] + sum(q(f"skip{l}.W")[s_][c] * g[c] for c in range(C))
                if l < a.n_layers - 1:
                    for c in range(C):
                        xn[t][c] = x[t][c] + q(f"res{l}.b")[c] + sum(q(f"res{l}.W")[c][k] * g[k] for k in range(C))
            x = xn
        skips.append(sk)
    z = []
    for t in range(T):
        cat = skips[0][t] + skips[1][t]
        h = [p["h1.b"][j] + sum(p["h1.W"][j][k] * max(cat[k], 0.0) for k in range(2 * S)) for j in range(H)]
        z.append(p["h2.b"][0] + sum(p["h2.W"][0][j] * h[j] for j in range(H)))
    return np.array(z)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_brute_force(seed):
    p = rand_params(TINY2, seed)
    u = np.random.default_rng(50 + seed).standard_normal((13, 2))
    assert np.allclose(forward_window(TINY2, p, u), brute_two_branch(TINY2, p, u), rtol=0, atol=1e-12)


def block_diagonal(a, p):
    """The single-trunk member (kind 1, channels 2C) whose weights are block-diagonal copies of the
    two branches, written out here slice by slice: branch b owns residual and skip channels
    [bC, (b+1)C) and, in each half of the dilated output, the same slice."""
    C, S = a.channels, a.skip_channels
    t = Arch(kind=1, in_channels=2, channels=2 * C, skip_channels=2 * S, head_channels=a.head_channels,
             n_stacks=a.n_stacks, layers_per_stack=a.layers_per_stack)
    q = {n: np.zeros(s) for n, s, _ in layout(t)}
    for b in range(2):
        r, sk = slice(b * C, (b + 1) * C), slice(b * S, (b + 1) * S)
        q["in.W"][r, b] = p[f"b{b}.in.W"][:, 0]
        q["in.b"][r] = p[f"b{b}.in.b"]
        for l in range(a.n_layers):
            for half in range(2):
                o = slice(half * 2 * C + b * C, half * 2 * C + (b + 1) * C)
                q[f"dil{l}.W"][o, r, :] = p[f"b{b}.dil{l}.W"][half * C:(half + 1) * C]
                q[f"dil{l}.b"][o] = p[f"b{b}.dil{l}.b"][half * C:(half + 1) * C]
            if l < a.n_layers - 1:
                q[f"res{l}.W"][r, r] = p[f"b{b}.res{l}.W"]
                q[f"res{l}.b"][r] = p[f"b{b}.res{l}.b"]
            q[f"skip{l}.W"][sk, r] = p[f"b{b}.skip{l}.W"]
            q[f"skip{l}.b"][sk] = p[f"b{b}.skip{l}.b"]
    for n in ("h1.W", "h1.b", "h2.W", "h2.b"):
        q[n] = p[n]
    return t, q


def test_block_diagonal_identity():
    a = Arch(kind=2, in_channels=2, channels=4, skip_channels=3, head_channels=5, n_stacks=2, layers_per_stack=3)
    p = rand_params(a, 9, 0.5)
    u = np.random.default_rng(9).standard_normal((2, 40, 2))
    t, q = block_diagonal(a, p)
    assert np.allclose(forward_window(a, p, u), forward_window(t, q, u), rtol=0, atol=1e-12)
    assert pack(t, q).size == num_params(t)


def test_branches_are_independent():
    p = rand_params(TINY2, 4)
    u = np.random.default_rng(4).standard_normal((30, 2))
    v = u.copy()
    v[7:, 1] += 1.0                                    # change the Livingston channel only
    cu, cv = [], []
    forward_window(TINY2, p, u, cu)
    forward_window(TINY2, p, v, cv)
    for a_, b_ in zip(cu, cv):
        if a_["branch"] == 0:
            assert np.array_equal(a_["skip"], b_["skip"])
        else:
            assert not np.allclose(a_["skip"], b_["skip"])
    p["h1.W"][:, TINY2.skip_channels:] = 0.0           # a head blind to the second branch
    assert np.array_equal(forward_window(TINY2, p, u), forward_window(TINY2, p, v))


def test_receptive_field_and_causality():
    a = Arch(kind=2, in_channels=2, channels=2, skip_channels=2, head_channels=2, n_stacks=2, layers_per_stack=3)
    rf = receptive_field(a)
    assert rf == 1 + 2 * (1 + 2 + 4)
    p = rand_params(a, 6)
    T = 40
    u = np.random.default_rng(6).standard_normal((T, 2))
    z = forward_window(a, p, u)
    t = 30

    def last_skip(x, br):        # the branch's final skip sum at t (before the head's ReLU)
        cap = []
        forward_window(a, p, x, cap)
        return [c["skip"] for c in cap if c["branch"] == br][-1][t]

    for ch in range(2):
        v = u.copy()
        v[t - rf + 1, ch] += 1.0
        assert np.all(last_skip(v, ch) != last_skip(u, ch))
        v = u.copy()
        v[t - rf, ch] += 1.0
        v[t + 1:, ch] += 3.0                           # the future does not matter either
        assert np.array_equal(last_skip(v, ch), last_skip(u, ch))
        assert forward_window(a, p, v)[t] == z[t]


def test_oracle_trunk_image_matches_slices():
    """The oracle's own block map gives the same trunk as the slice-by-slice statement above."""
    from oracle.arch import two_branch_as_trunk
    a = Arch(kind=2, in_channels=2, channels=3, skip_channels=2, head_channels=4, n_stacks=1, layers_per_stack=3)
    p = rand_params(a, 12)
    t1, q1 = block_diagonal(a, p)
    t2, q2 = two_branch_as_trunk(a, p)
    assert t1 == t2
    assert all(np.array_equal(q1[n], q2[n]) for n in q1)


def test_gradient_by_central_differences():
    """The two-branch gradient (the trunk's reverse mode read back through the block map) against
    central differences of the two-branch forward itself, every parameter of a tiny member."""
    from oracle.arch import pack
    from oracle.train import loss_and_grad, loss_only
    a = Arch(kind=2, in_channels=2, channels=2, skip_channels=2, head_channels=3, n_stacks=1, layers_per_stack=3,
             head_mid_relu=1)
    rng = np.random.default_rng(3)
    blob = pack(a, rand_params(a, 13, 0.6))
    u = rng.standard_normal((2, 20, 2))
    y = (rng.uniform(size=(2, 20)) < 0.3).astype(float)
    loss, g, du = loss_and_grad(a, blob, u, y)
    assert abs(loss - loss_only(a, blob, u, y)) < 1e-14
    h = 1e-6
    fd = np.empty_like(blob)
    for i in range(blob.size):
        e = np.zeros_like(blob)
        e[i] = h
        fd[i] = (loss_only(a, blob + e, u, y) - loss_only(a, blob - e, u, y)) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-7 * max(1.0, np.max(np.abs(g)))
    # the input gradient as well (two channels, each through its own branch)
    fdu = np.empty_like(u)
    for idx in np.ndindex(u.shape):
        e = np.zeros_like(u)
        e[idx] = h
        fdu[idx] = (loss_only(a, blob, u + e, y) - loss_only(a, blob, u - e, y)) / (2 * h)
    assert np.max(np.abs(fdu - du)) < 1e-7 * max(1.0, np.max(np.abs(du)))

