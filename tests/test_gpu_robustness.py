"""Device-level properties that hold at any size and catch whole classes of kernel mistakes:
- causality ("AI architecture": causal convolutions): perturbing a stream after sample p leaves every
  ensemble score before p, and every per-window logit before it, bit for bit unchanged, in every
  precision and through every fused launch (history rows, chunk edges, sub-sequence interleaving);
- guard bands: the kernels write inside their output buffers only (NaN-patterned bands around each
  output are bit for bit intact afterwards, and the output holds no NaN), the persistent forward
  included;
- checkpoint and resume of training: two steps, a checkpoint, a fresh model and trainer from it and
  one more step give the same master weights, moments and loss, bit for bit, as three steps without
  interruption."""
import numpy as np
import pytest

from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GUARD = 4096
PATTERN = 0x7FC0BEEF   # a quiet-NaN bit pattern no kernel writes


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_11133_amd import gwd
    return gwd


def guarded(n, dtype=torch.float32):
    """A device buffer of n elements between two guard bands filled with PATTERN (per 32-bit word)."""
    es = torch.empty((), dtype=dtype).element_size()
    words = (n * es + 2 * GUARD * 4) // 4
    buf = torch.full((words,), PATTERN, dtype=torch.int32, device="cuda")
    body = buf[GUARD:GUARD + n * es // 4].view(dtype)
    return buf, body


def guards_intact(buf, n_body_words):
    head = buf[:GUARD]
    tail = buf[GUARD + n_body_words:]
    return bool((head == PATTERN).all()) and bool((tail == PATTERN).all())


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_causality_of_the_stitched_scores(g, prec):
    from paper_2201_11133_amd import synth
    print(f"case: causality {prec}", flush=True)
    W, S = 4096, 256
    blobs = np.stack([synth.full_weights(31), synth.full_weights(32)])
    m = g.Model(g.full_arch(), blobs, prec)
    x, _ = synth.make_stream(400, 6.0, 1)
    rng = np.random.default_rng(401)
    for p in (13_001, 4096 * 3 + 17):
        x2 = x.copy()
        x2[p:] = rng.standard_normal(x2[p:].shape).astype(np.float32)
        e1 = m.forward([to_dev(x)], W, S, out_mode=1).clone()
        e2 = m.forward([to_dev(x2)], W, S, out_mode=1).clone()
        L = x.shape[0]
        for k in range(3):   # the ensemble score, then each member's stitched logits
            a, b = e1[k * L:(k + 1) * L], e2[k * L:(k + 1) * L]
            assert torch.equal(a[:p], b[:p]), (prec, p, k)
            assert not torch.equal(a[p:], b[p:])
        # per-window logits: window j is unchanged at positions before p - j S
        w1 = m.forward([to_dev(x)], W, S, out_mode=2).view(2, -1, W)
        w2 = m.forward([to_dev(x2)], W, S, out_mode=2).view(2, -1, W)
        for j in range(w1.shape[1]):
            q = min(max(p - j * S, 0), W)
            assert torch.equal(w1[:, j, :q], w2[:, j, :q]), (prec, p, j)
    m.close()


def test_causality_small_member(g):
    from paper_2201_11133_amd import synth
    print("case: causality, small member", flush=True)
    m = g.Model(g.tiny_arch(), synth.tiny_weights(3), "fp32")
    x, _ = synth.make_stream(402, 3.0, 0)
    p = 7_777
    x2 = x.copy()
    x2[p:] *= -3.0
    e1 = m.forward([to_dev(x)], 4096, 256, out_mode=0)
    e2 = m.forward([to_dev(x2)], 4096, 256, out_mode=0)
    assert torch.equal(e1[:p], e2[:p]) and not torch.equal(e1[p:], e2[p:])
    m.close()


@pytest.mark.parametrize("prec,mode,persistent", [("bf16", 0, False), ("bf16", 1, False), ("bf16", 2, False),
                                                  ("fp8", 2, False), ("fp32", 0, False), ("bf16", 1, True),
                                                  ("fp8", 2, True)])
def test_forward_writes_inside_its_output(g, prec, mode, persistent):
    from paper_2201_11133_amd import synth
    print(f"case: guard bands forward {prec} mode {mode}{' persistent' if persistent else ''}", flush=True)
    W, S = 4096, 256
    blobs = np.stack([synth.full_weights(33), synth.full_weights(34)])
    m = g.Model(g.full_arch(), blobs, prec)
    if persistent:
        m.set_persistent(True)
    xs = [to_dev(synth.make_stream(403, 5.3, 1)[0]), to_dev(synth.make_stream(404, 0.7, 0)[0])]
    n = m.out_floats(xs, W, S, mode)
    buf, out = guarded(n)
    m.forward(xs, W, S, out_mode=mode, out=out)
    torch.cuda.synchronize()
    assert guards_intact(buf, n)
    assert bool(torch.isfinite(out).all())
    m.close()


def test_slide_and_whitening_write_inside_their_outputs(g):
    from paper_2201_11133_amd import synth
    print("case: guard bands, time slide and whitening", flush=True)
    L, nps = 1 << 16, 4096
    src = to_dev(synth.coloured_stream(405, L))
    shifts = [0, 4096 * 3, -77]
    buf, out = guarded(len(shifts) * L * 2)
    g.time_slide(src, shifts, out=out.view(len(shifts), L, 2))
    pbuf, psd = guarded(2 * (nps // 2 + 1), torch.float64)
    g.welch_psd(src, nps, 4096.0, out=psd.view(2, nps // 2 + 1))
    wbuf, y = guarded(L * 2)
    g.whiten(src, psd.view(2, nps // 2 + 1), nps, 4096.0, True, out=y.view(L, 2))
    torch.cuda.synchronize()
    assert guards_intact(buf, len(shifts) * L * 2)
    assert guards_intact(pbuf, 2 * (nps // 2 + 1) * 2)
    assert guards_intact(wbuf, L * 2)
    assert bool(torch.isfinite(out).all()) and bool(torch.isfinite(psd).all()) and bool(torch.isfinite(y).all())


def test_checkpoint_resume_is_exact(g, tmp_path):
    from paper_2201_11133_amd import synth
    print("case: training checkpoint and resume", flush=True)
    B, T = 4, 4096
    blob = synth.full_weights(35)
    x, injs = synth.make_windows(406, B, B // 2)
    y = np.zeros((B, T), np.float32)
    for i, inj in injs:
        y[i] = synth.box_labels(T, inj.tc)
    xd, yd = to_dev(x), to_dev(y)
    # three steps without interruption
    m = g.Model(g.full_arch(), blob, "bf16")
    tr = g.Trainer(m, blob, B, T)
    losses = [float(tr.step(xd, yd)[0].item()) for _ in range(3)]
    ref = [t.cpu().clone() for t in (tr.master, tr.mom, tr.vel)]
    m.close()
    # two steps, a checkpoint, then a fresh trainer from it
    m = g.Model(g.full_arch(), blob, "bf16")
    tr = g.Trainer(m, blob, B, T)
    for _ in range(2):
        tr.step(xd, yd)
    path = str(tmp_path / "ckpt.safetensors")
    tr.save(path)
    m.close()
    tr2 = g.Trainer.resume(path)
    assert tr2.step_no == 2
    loss3 = float(tr2.step(xd, yd)[0].item())
    assert loss3 == losses[2]
    for a, b in zip(ref, (tr2.master, tr2.mom, tr2.vel)):
        assert torch.equal(a, b.cpu())
    tr2.m.close()
