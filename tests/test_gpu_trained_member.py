"""A member trained by this package's own training path (BF16 forward and backward, Adam on fp32
master weights, 300 steps of batch 256 x 4096 on fresh synthetic batches, half of them chirped,
labels 1 within 0.1 s of the coalescence time): its BCE loss falls, and the reduced-precision error
against the FP64 oracle on the trained weights meets the 2e-2 target for BF16 (on random He-normal
weights it does not: rounding is amplified through 30 layers). FP8's error is stated. Training is
deterministic, so the trained weights, and these figures, are the same on every run."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STEPS, LR, B, T = 300, 1e-3, 256, 4096


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_11133_amd import gwd
    return gwd


@pytest.mark.timeout(900)
def test_trained_member_reduced_precision_error(g):
    from oracle.arch import FULL, unpack
    from oracle.forward import forward_window, sigmoid
    from oracle.stream import gather_windows
    from paper_2201_11133_amd import synth
    print(f"case: train {STEPS} steps, then reduced-precision error", flush=True)
    blob = synth.full_weights(4)
    m = g.Model(g.full_arch(), blob, "bf16")
    tr = g.Trainer(m, blob, B, T)
    losses = []
    for step in range(STEPS):
        x, injs = synth.make_windows(5000 + step, B, B // 2)
        y = np.zeros((B, T), np.float32)
        for i, inj in injs:
            y[i] = synth.box_labels(T, inj.tc)
        loss, _ = tr.step(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), lr=LR)
        losses.append(float(loss.item()))
        if step % 50 == 0:
            print(f"  step {step}: loss {losses[-1]:.4f}", flush=True)
    w = tr.master.cpu().numpy()
    m.close()
    print(f"loss: first {losses[0]:.4f}, mean of the last 20 {np.mean(losses[-20:]):.4f}", flush=True)
    assert np.mean(losses[-20:]) < 0.5 * losses[0]
    xs, _ = synth.make_stream(777, (4096 + 7 * 256) / 4096, 1)
    win = gather_windows(xs.astype(np.float64), 4096, 256)
    p64 = sigmoid(forward_window(FULL, unpack(FULL, w.astype(np.float64)), win))
    err = {}
    for prec in ("fp32", "bf16", "fp8"):
        mm = g.Model(g.full_arch(), w, prec)
        z = mm.forward([torch.from_numpy(xs).cuda()], 4096, 256, out_mode=2).cpu().numpy().reshape(-1, 4096)
        mm.close()
        dp = np.abs(sigmoid(z.astype(np.float64)) - p64)
        err[prec] = (float(dp.max()), float(dp.mean()))
        print(f"trained member {prec}: max|dp| = {dp.max():.3g}, mean {dp.mean():.3g} (8 windows)", flush=True)
    assert err["fp32"][0] <= 1e-5
    assert err["bf16"][0] <= 2e-2
