"""Captured plans (one graph launch for all members and ragged streams), tiling choices, autotuner."""
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


def ragged_streams(seed, n, max_s=40.0):
    from paper_2201_11133_amd import synth
    rng = np.random.default_rng(seed)
    lens = [int(4096 * np.exp(rng.uniform(np.log(0.5), np.log(max_s)))) for _ in range(n)]
    lens[1] = 0        # an empty stream
    lens[2] = 3000     # shorter than one window
    return [synth.make_stream(seed + i, max(L, 1) / 4096, 1 if L > 16 * 4096 else 0)[0][:L] for i, L in enumerate(lens)]


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_plan_replays_match_eager(g, prec):
    from paper_2201_11133_amd import synth
    print(f"case: plan replays {prec}", flush=True)
    blobs = np.stack([synth.full_weights(11 + i) for i in range(2)])
    m = g.Model(g.full_arch(), blobs, prec)
    m.set_tiling(0, 0, 96)       # several batches, streams split across batch boundaries
    xs = ragged_streams(300, 6)
    bufs = [to_dev(x) if len(x) else torch.zeros((0, 2), dtype=torch.float32, device="cuda") for x in xs]
    plan = m.plan(bufs, 4096, 256, out_mode=1)
    for rep in range(3):
        # new data in the same buffers, then eager work between replays
        for b in bufs:
            if b.numel():
                b.copy_(torch.randn_like(b))
        eager = m.forward(bufs, 4096, 256, out_mode=1).clone()
        torch.cuda.synchronize()
        got = plan.launch().clone()
        torch.cuda.synchronize()
        assert torch.equal(got, eager), rep
    per, tot = plan.completion_us()
    lens = [len(x) for x in xs]
    assert tot > 0 and np.all(per <= tot + 1e-6)
    assert all((p > 0) == (L > 0) for p, L in zip(per, lens))
    plan.close()
    m.close()


TILINGS = [(64, 4), (64, 8), (128, 4)]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_tilings_and_batches_do_not_change_results(g, prec):
    """Every schedule (tiling, fused triples or one layer per launch, batch size) computes each
    output with the same operations in the same order: results are bit-identical."""
    from paper_2201_11133_amd import synth
    print(f"case: schedules {prec}", flush=True)
    m = g.Model(g.full_arch(), synth.full_weights(11), prec)
    # a long stream, one shorter than a window, one that ends inside its last window
    xs = [to_dev(synth.make_stream(310, 20.0, 1)[0]), to_dev(synth.make_stream(311, 0.6, 0)[0]),
          to_dev(synth.make_stream(312, 3.3, 0)[0][: 3 * 4096 + 1234])]
    ref = None
    fuses = (1, 3, 6)   # one layer, triples and quads, sextets and quads per launch
    for fuse in fuses:
        for rows, waves in TILINGS:
            for nb in (7, 64, 300, 512):
                m.set_tiling(rows, waves, nb, fuse)
                e = m.forward(xs, 4096, 256, 1).clone()
                if ref is None:
                    ref = e
                assert torch.equal(e, ref), (fuse, rows, waves, nb)
    # fused launches aiming at more blocks: more segments per sub-sequence, each after a warm-up chunk
    for blocks in (1024, 2048, 8192):
        m.set_fused_blocks(blocks)
        for nb in (64, 512):
            for fuse in fuses[1:]:
                m.set_tiling(64, 4, nb, fuse)
                assert torch.equal(m.forward(xs, 4096, 256, 1), ref), (blocks, nb, fuse)
    m.set_fused_blocks(0)
    m.close()


def test_layers_per_launch_values(g):
    """gwd_set_tiling: six layers per launch (sextets and quads) for gated BF16/FP8 models with stacks
    of ten layers, the default there; FP32 and the small member refuse fused schedules."""
    from paper_2201_11133_amd import synth
    print("case: layers per launch values", flush=True)
    for prec in ("bf16", "fp8"):
        m = g.Model(g.full_arch(), synth.full_weights(13), prec)
        assert m.fused_layers(0, 4096) == 6 and m.fused_layers(6, 4096) == 4 and m.fused_layers(3, 4096) == 0
        m.set_tiling(0, 0, 512, 3)
        assert m.fused_layers(0, 4096) == 3 and m.fused_layers(3, 4096) == 3 and m.fused_layers(6, 4096) == 4
        assert m.fused_layers(6, 8192) == 3     # triples and quads: the quad needs one-chunk sub-sequences
        m.set_tiling(0, 0, 512, 6)
        assert m.fused_layers(6, 8192) == 4     # sextets and quads: quads at any window length
        assert g.lib.gwd_set_tiling(m.h, 0, 0, 5, 512) == g.ERR_ARG
        m.set_tiling()
        assert m.fused_layers(0, 4096) == 6
        m.close()
    m = g.Model(g.full_arch(), synth.full_weights(13), "fp32")
    assert g.lib.gwd_set_tiling(m.h, 0, 0, 6, 512) == g.ERR_ARG
    assert g.lib.gwd_set_tiling(m.h, 0, 0, 3, 512) == g.ERR_ARG
    m.close()
    m = g.Model(g.tiny_arch(), synth.tiny_weights(3), "bf16")
    assert g.lib.gwd_set_tiling(m.h, 0, 0, 6, 512) == g.ERR_ARG
    m.close()


def test_autotune_picks_a_valid_tiling(g, tmp_path, monkeypatch):
    from paper_2201_11133_amd import synth
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("GWD_AUTOTUNE_CACHE", str(cache))
    m = g.Model(g.full_arch(), synth.full_weights(11), "bf16")
    x = to_dev(synth.make_stream(311, 40.0, 1)[0])
    rw, w, fu, b, fb, pe = m.autotune([x])
    assert (rw, w) in TILINGS and fu in (1, 3, 6) and b in (256, 512, 1024) and pe in (0, 1)
    if pe:    # the persistent forward: fused layers (sextets and quads here), one launch
        assert fu == 6 and fb == 0 and b == 512
    else:
        assert fb in ((512, 1024, 2048) if fu == 3 else (512, 1024) if fu == 6 else (0,))
    assert cache.read_text().strip().endswith(f"{rw} {w} {fu} {b} {fb} {pe}")
    print(f"autotuned: rows {rw}, waves {w}, layers per launch {fu}, batch {b}, fused blocks {fb}, "
          f"persistent {pe}", flush=True)
    # second call reads the cache
    assert m.autotune([x]) == (rw, w, fu, b, fb, pe)
    m.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_long_windows_give_the_same_scores(g, prec):
    """Stitched scores depend only on each owned row's receptive field (W - S >= RF - 1), and every row
    is computed with the same operations wherever it sits in a window: windows of 2^16 samples with
    stride 2^16 - 3072 give bit-identical ensemble scores to windows of 4096 with stride 256."""
    from paper_2201_11133_amd import synth
    print(f"case: long windows {prec}", flush=True)
    blobs = np.stack([synth.full_weights(11 + i) for i in range(2)])
    m = g.Model(g.full_arch(), blobs, prec)
    xs = [to_dev(synth.make_stream(320, 40.0, 2)[0]), to_dev(synth.make_stream(321, 3.7, 0)[0])]
    a = m.forward(xs, 4096, 256, 1).clone()
    W = 1 << 16
    b = m.forward(xs, W, W - 3072, 1).clone()
    assert torch.equal(a, b)
    m.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("W,S", [(3200, 128), (3328, 200)])
def test_fused_triples_with_partial_chunks(g, prec, W, S):
    """Windows whose interleaved sub-sequences end inside a chunk (W = 3200: 50 rows at dilation 64,
    400 at dilation 8; W = 3328: 52 and 416) and strides that are not multiples of a chunk: fused
    triples give the same outputs as one layer per launch, per window (out_mode 2) and stitched."""
    from paper_2201_11133_amd import synth
    print(f"case: partial chunks {prec} W={W} S={S}", flush=True)
    m = g.Model(g.full_arch(), synth.full_weights(12), prec)
    xs = [to_dev(synth.make_stream(330, 6.0, 1)[0]), to_dev(synth.make_stream(331, 1.1, 0)[0][:4321])]
    res = {}
    fuses = (1, 3, 6)
    for fuse in fuses:
        m.set_tiling(0, 0, 64, fuse)
        res[fuse] = (m.forward(xs, W, S, 2).clone(), m.forward(xs, W, S, 1).clone())
    for fuse in fuses[1:]:
        assert torch.equal(res[1][0], res[fuse][0]), fuse
        assert torch.equal(res[1][1], res[fuse][1]), fuse
    m.close()
