"""The two-branch member (one gated branch per detector, Fig. 1) on the GPU: the weights the library
runs equal the block-diagonal image of the branches (bit for bit, fp32; quantised like any trunk for
BF16 / FP8), FP32 logits match the oracle's branch-by-branch forward, and the reduced-precision error
is stated. Training is refused."""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import FP32_P_TOL, sigmoid64, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_11133_amd import gwd
    return gwd


@pytest.fixture(scope="module")
def blob():
    from paper_2201_11133_amd import synth
    return synth.two_branch_weights(21)


@pytest.fixture(scope="module")
def dense(blob):
    """The oracle's branch parameters and the block-diagonal trunk they equal (test-side statement)."""
    from oracle.arch import TWO_BRANCH, unpack
    from tests.test_oracle_two_branch import block_diagonal
    p = unpack(TWO_BRANCH, blob.astype(np.float64))
    t, q = block_diagonal(TWO_BRANCH, p)
    return p, t, q


def test_export_is_the_block_diagonal_image(g, blob, dense):
    from oracle.arch import pack
    print("case: two-branch export fp32", flush=True)
    _, t, q = dense
    m = g.Model(g.two_branch_arch(), blob, "fp32")
    assert np.array_equal(m.export_weights(0), pack(t, q).astype(np.float32))
    m.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_export_quantised(g, blob, dense, prec):
    """The expanded trunk is quantised exactly like any trunk: the oracle quantisers applied to the
    block-diagonal matrices give the exported operands (the zero blocks stay zero)."""
    from oracle.arch import unpack
    from tests.test_gpu_lowp import quantised_layer_mats
    print(f"case: two-branch export {prec}", flush=True)
    _, t, q = dense
    m = g.Model(g.two_branch_arch(), blob, prec)
    pe = unpack(t, m.export_weights(0).astype(np.float64))
    for l in (0, 13, 29):
        last = l == 29
        Bc, sc, Brs, srs = quantised_layer_mats(prec, q, l, last)
        We = pe[f"dil{l}.W"]
        Bce = np.concatenate([We[:, :, 0].T, We[:, :, 1].T], axis=0)
        assert np.array_equal(Bce, (Bc * sc[None, :]).astype(np.float32).astype(np.float64))
        Brse = pe[f"skip{l}.W"].T if last else np.concatenate([pe[f"res{l}.W"].T, pe[f"skip{l}.W"].T], axis=1)
        assert np.array_equal(Brse, (Brs * srs[None, :]).astype(np.float32).astype(np.float64))
        assert np.all(We[:64, 64:] == 0) and np.all(We[64:128, :64] == 0)     # off-diagonal blocks
    m.close()


def test_fp32_windows_and_stitched_slice(g, blob, dense):
    """Per-window logits of a ragged 8-window stream and the stitched scores of a 16 s slice with a
    chirp, against the oracle's two-branch forward."""
    from oracle.arch import TWO_BRANCH
    from oracle.forward import forward_stream, forward_window
    from oracle.stream import gather_windows
    from paper_2201_11133_amd import synth
    print("case: two-branch fp32 parity", flush=True)
    p, _, _ = dense
    m = g.Model(g.two_branch_arch(), blob, "fp32")
    W, S = 4096, 256
    L = W + 6 * S + 100
    x, _ = synth.make_stream(305, L / 4096, 0)
    z2 = m.forward([to_dev(x)], W, S, out_mode=2).cpu().numpy().reshape(-1, W)
    zw = forward_window(TWO_BRANCH, p, gather_windows(x.astype(np.float64), W, S))
    dp = np.abs(sigmoid64(z2) - sigmoid64(zw)).max()
    print(f"  two-branch fp32 per-window max|dp| = {dp:.3g}", flush=True)
    assert dp <= FP32_P_TOL
    xs, _ = synth.make_stream(306, 16.0, 1)
    e = m.forward([to_dev(xs)], W, S, out_mode=0).cpu().numpy()
    z64 = forward_stream(TWO_BRANCH, p, xs.astype(np.float64))
    dps = np.abs(sigmoid64(e) - sigmoid64(z64)).max()
    print(f"  two-branch fp32 16 s slice max|dp| = {dps:.3g}", flush=True)
    assert dps <= FP32_P_TOL
    m.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_low_precision_error_stated(g, blob, dense, prec):
    """End-to-end probability error of the reduced-precision two-branch member on 4 windows against
    the FP64 oracle (stated; the layer kernels are those of the trunk, whose layer-local parity is
    gated elsewhere)."""
    from oracle.arch import TWO_BRANCH
    from oracle.forward import forward_window
    from paper_2201_11133_amd import synth
    print(f"case: two-branch {prec} stated error", flush=True)
    p, _, _ = dense
    x, _ = synth.make_windows(307, 4, 2)
    m = g.Model(g.two_branch_arch(), blob, prec)
    z = m.forward([to_dev(x[i]) for i in range(4)], 4096, 256, out_mode=2).cpu().numpy().reshape(4, -1)
    z64 = forward_window(TWO_BRANCH, p, x.astype(np.float64))
    dp = np.abs(sigmoid64(z) - sigmoid64(z64))
    print(f"  two-branch {prec}: max|dp| {dp.max():.3g}, mean {dp.mean():.3g}", flush=True)
    assert np.all(np.isfinite(z))
    m.close()


def test_training_is_refused(g, blob):
    m = g.Model(g.two_branch_arch(), blob, "bf16")
    B, W = 2, 4096
    w = torch.zeros((B, W, 2), dtype=torch.float32, device="cuda")
    z = torch.zeros((B, W), dtype=torch.float32, device="cuda")
    rc = g.lib.gwd_forward_train(m.h, 0, w.data_ptr(), B, W, z.data_ptr(), z.data_ptr(), None)
    assert rc == g.ERR_UNSUPPORTED
    m.close()


def test_zero_block_skipping_is_exact(g, dense):
    """BF16: the two-branch model's fused kernels take only each wave's own group of k-steps; a kind-1
    model loaded with the same block-diagonal weights runs every step. The skipped steps add exact
    zero products, so the scores (ensemble and per member) are identical."""
    from oracle.arch import pack
    from paper_2201_11133_amd import synth
    from oracle.arch import TWO_BRANCH, unpack
    from tests.test_oracle_two_branch import block_diagonal
    print("case: two-branch zero-block skipping vs dense trunk", flush=True)
    blobs = np.stack([synth.two_branch_weights(40 + i) for i in range(2)])
    trunk = np.stack([pack(*block_diagonal(TWO_BRANCH, unpack(TWO_BRANCH, b.astype(np.float64)))).astype(np.float32)
                      for b in blobs])
    x, _ = synth.make_stream(308, 64.0, 2)
    xd = to_dev(x)
    m2 = g.Model(g.two_branch_arch(), blobs, "bf16")
    m1 = g.Model(g.full_arch(), trunk, "bf16")
    a = m2.forward([xd], 4096, 256, out_mode=1).cpu().numpy()
    b = m1.forward([xd], 4096, 256, out_mode=1).cpu().numpy()
    assert np.array_equal(a, b)
    m2.close()
    m1.close()
