"""Pins for the oracle gradient (FP64 central finite differences, linear closed form) and Adam."""
import numpy as np
import pytest

from oracle.arch import TINY, Arch, num_params, unpack
from oracle.train import adam_step, bce_grad, bce_logits, loss_and_grad, loss_only
from paper_2201_11133_amd import synth

SMALL1 = Arch(kind=1, in_channels=2, channels=3, skip_channels=4, head_channels=3,
              n_stacks=2, layers_per_stack=3, kernel_size=2, input_kernel=1, head_mid_relu=0)
SMALL1_MID = Arch(**{**SMALL1.__dict__, "head_mid_relu": 1})
SMALL1_K2 = Arch(**{**SMALL1.__dict__, "input_kernel": 2})


def test_bce_definition():
    z = np.array([-3.0, 0.0, 2.0, 40.0, -40.0])
    y = np.array([0.0, 1.0, 1.0, 0.0, 1.0])
    ref = np.mean(np.log1p(np.exp(z)) - y * z)
    assert abs(bce_logits(z, y) - ref) < 1e-12
    # derivative of the mean loss w.r.t. each logit, by central differences
    h = 1e-6
    for i in range(z.size):
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        fd = (bce_logits(zp, y) - bce_logits(zm, y)) / (2 * h)
        assert abs(fd - bce_grad(z, y)[i]) < 1e-8


def _fd_check(a, blob, u, y, idx, h=1e-6, rtol=1e-5, atol=1e-9):
    _, g, _ = loss_and_grad(a, blob, u, y)
    for i in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss_only(a, bp, u, y) - loss_only(a, bm, u, y)) / (2 * h)
        assert abs(fd - g[i]) <= atol + rtol * abs(fd), (i, fd, g[i])
    return g


@pytest.mark.parametrize("a", [SMALL1, SMALL1_MID, SMALL1_K2], ids=["kind1", "kind1_midrelu", "kind1_inkernel2"])
def test_gradient_fd_small_gated(a):
    rng = np.random.default_rng(0)
    blob = rng.standard_normal(num_params(a)) * 0.6
    u = rng.standard_normal((2, 40, 2))
    y = (rng.uniform(size=(2, 40)) < 0.3).astype(float)
    _fd_check(a, blob, u, y, range(num_params(a)))


def test_gradient_fd_tiny_member():
    """FP64 central differences, h = 1e-6, on the tiny member (all 1,681 parameters on a short batch)."""
    blob = synth.tiny_weights(0).astype(np.float64)
    u, injs = synth.make_windows(100, 2, 1, W=256)
    u = u.astype(np.float64)
    y = np.zeros((2, 256))
    y[:, 100:140] = 1.0
    _fd_check(TINY, blob, u, y, range(num_params(TINY)), rtol=1e-4, atol=1e-10)


def test_input_gradient_fd():
    rng = np.random.default_rng(1)
    a = SMALL1
    blob = rng.standard_normal(num_params(a)) * 0.6
    u = rng.standard_normal((1, 30, 2))
    y = (rng.uniform(size=(1, 30)) < 0.5).astype(float)
    _, _, du = loss_and_grad(a, blob, u, y)
    h = 1e-6
    for t in [0, 7, 29]:
        for c in range(2):
            up, um = u.copy(), u.copy()
            up[0, t, c] += h
            um[0, t, c] -= h
            fd = (loss_only(a, blob, up, y) - loss_only(a, blob, um, y)) / (2 * h)
            assert abs(fd - du[0, t, c]) <= 1e-9 + 1e-5 * abs(fd)


def test_linear_closed_form_tiny():
    """All biases large so every ReLU is active: the tiny member is linear in u, and the
    gradient of the loss w.r.t. the output bias is the mean of (sigmoid(z) - y) exactly."""
    rng = np.random.default_rng(2)
    p = unpack(TINY, synth.tiny_weights(0).astype(np.float64))
    blob = synth.tiny_weights(0).astype(np.float64)
    n = num_params(TINY)
    # raise conv biases (entries that are biases in blob order) so pre-activations stay positive
    off = 0
    from oracle.arch import layout
    for name, shape, fan in layout(TINY):
        cnt = int(np.prod(shape))
        if name.startswith("conv") and name.endswith(".b"):
            blob[off:off + cnt] = 200.0
        off += cnt
    u = rng.standard_normal((1, 64, 2)) * 0.1
    y = np.zeros((1, 64))
    loss, g, _ = loss_and_grad(TINY, blob, u, y)
    from oracle.forward import forward_window, sigmoid
    z = forward_window(TINY, unpack(TINY, blob), u)
    assert abs(g[n - 1] - np.mean(sigmoid(z) - y)) < 1e-12
    # linearity in u for the input gradient: d z / d u does not depend on u
    _, _, du1 = loss_and_grad(TINY, blob, u, y)
    assert np.all(np.isfinite(du1))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    w = rng.standard_normal(1000)
    g = rng.standard_normal(1000) * 10 ** rng.uniform(-6, 2, 1000)
    lr, eps = 1e-3, 1e-8
    w1, m, v = adam_step(w, g, np.zeros(1000), np.zeros(1000), 1, lr=lr, eps=eps)
    np.testing.assert_allclose(w1 - w, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_second_step():
    w = np.array([1.0])
    g1, g2 = np.array([0.5]), np.array([-0.25])
    w1, m, v = adam_step(w, g1, np.zeros(1), np.zeros(1), 1)
    w2, m, v = adam_step(w1, g2, m, v, 2)
    m_ref = 0.9 * 0.1 * 0.5 + 0.1 * -0.25
    v_ref = 0.999 * 0.001 * 0.25 + 0.001 * 0.0625
    step = 1e-3 * (m_ref / (1 - 0.81)) / (np.sqrt(v_ref / (1 - 0.999 ** 2)) + 1e-8)
    assert abs(w2[0] - (w1[0] - step)) < 1e-15
