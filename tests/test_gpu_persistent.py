"""The persistent forward (gwd_set_persistent): one launch for every member and every window of
ragged streams, each block owning a window at a time. Its scores must equal the launch sequence's
bit for bit (the same layer bodies in the same order), in every output mode and precision, eagerly
and inside a captured plan; plans report a completion time per stream from the kernel itself."""
import numpy as np
import pytest

from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_11133_amd import gwd
    return gwd


def ragged(seed, n, max_s=24.0):
    """n streams of log-uniform length (one empty, one shorter than a window), as device buffers."""
    from paper_2201_11133_amd import synth
    rng = np.random.default_rng(seed)
    lens = [int(4096 * np.exp(rng.uniform(np.log(0.5), np.log(max_s)))) for _ in range(n)]
    lens[1] = 0
    lens[2] = 3000
    xs = [synth.make_stream(seed + i, max(L, 1) / 4096, 1 if L > 8 * 4096 else 0)[0][:L] for i, L in enumerate(lens)]
    return lens, [to_dev(x) if len(x) else torch.zeros((0, 2), dtype=torch.float32, device="cuda") for x in xs]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_persistent_equals_launch_sequence(g, prec, mode):
    from paper_2201_11133_amd import synth
    print(f"case: persistent {prec} out_mode {mode}", flush=True)
    blobs = np.stack([synth.full_weights(61 + i) for i in range(3)])
    m = g.Model(g.full_arch(), blobs, prec)
    _, bufs = ragged(700 + mode, 7)
    ref = m.forward(bufs, 4096, 256, out_mode=mode).clone()
    m.set_persistent(True)
    got = m.forward(bufs, 4096, 256, out_mode=mode).clone()
    again = m.forward(bufs, 4096, 256, out_mode=mode).clone()
    m.set_persistent(False)
    back = m.forward(bufs, 4096, 256, out_mode=mode).clone()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(ref).all())
    assert torch.equal(got, ref) and torch.equal(again, ref) and torch.equal(back, ref)
    m.close()


def test_persistent_plan_and_completion_times(g):
    from paper_2201_11133_amd import synth
    print("case: persistent plan", flush=True)
    blobs = np.stack([synth.full_weights(71 + i) for i in range(2)])
    m = g.Model(g.full_arch(), blobs, "bf16")
    lens, bufs = ragged(710, 9, 40.0)
    m.set_persistent(True)
    plan = m.plan(bufs, 4096, 256, out_mode=1)
    for rep in range(3):
        for b in bufs:   # new data in the same buffers, eager work between replays
            if b.numel():
                b.copy_(torch.randn_like(b))
        m.set_persistent(False)
        eager = m.forward(bufs, 4096, 256, out_mode=1).clone()
        m.set_persistent(True)
        torch.cuda.synchronize()
        got = plan.launch().clone()
        torch.cuda.synchronize()
        assert torch.equal(got, eager), rep
    per, tot = plan.completion_us()
    assert tot > 0 and np.all(per <= tot + 1e-6)
    assert all((p > 0) == (L > 0) for p, L in zip(per, lens))
    plan.close()
    m.close()


def test_persistent_needs_fused_layers(g):
    from paper_2201_11133_amd import synth
    print("case: persistent, unsupported requests", flush=True)
    m = g.Model(g.full_arch(), synth.full_weights(72)[None], "fp32")
    with pytest.raises(RuntimeError):
        m.set_persistent(True)
    m.close()
    m = g.Model(g.full_arch(), synth.full_weights(72)[None], "bf16")
    assert g.lib.gwd_set_persistent(m.h, 2) == g.ERR_ARG
    m.set_persistent(True)
    x = to_dev(synth.make_stream(711, 6.0, 0)[0])
    with pytest.raises(RuntimeError):   # windows of 8192: the last layer of a stack is a single launch
        m.forward([x], 8192, 4096, out_mode=0)
    m.set_tiling(64, 4, 512, 1)        # one layer per launch: not a persistent form
    with pytest.raises(RuntimeError):
        m.forward([x], 4096, 256, out_mode=0)
    m.close()
