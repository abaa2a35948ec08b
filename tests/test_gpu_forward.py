"""GPU parity of the forward path (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

from tests.gpu_common import FP32_P_TOL, U32, sigmoid64, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_11133_amd import gwd
    return gwd


@pytest.fixture(scope="module")
def full_blob():
    from paper_2201_11133_amd import synth
    return synth.full_weights(1)


@pytest.fixture(scope="module")
def full_model(g, full_blob):
    m = g.Model(g.full_arch(), full_blob, "fp32")
    yield m
    m.close()


def oracle_params(blob, arch="full", mid=0):
    from oracle.arch import FULL, TINY, Arch, unpack
    a = TINY if arch == "tiny" else Arch(**{**FULL.__dict__, "head_mid_relu": mid})
    return a, unpack(a, blob.astype(np.float64))


# ---------------------------------------------------------------- weights
def test_export_is_exact_fp32(g, full_model, full_blob):
    print("case: export fp32 full", flush=True)
    assert np.array_equal(full_model.export_weights(0), full_blob)


def test_export_tiny(g):
    from paper_2201_11133_amd import synth
    blob = synth.tiny_weights(0)
    m = g.Model(g.tiny_arch(), blob, "fp32")
    assert np.array_equal(m.export_weights(0), blob)
    m.close()


# ---------------------------------------------------------------- tiny member (64 windows, 8 chirped)
def test_tiny_member_parity_and_triggers(g):
    from oracle.forward import forward_window
    from paper_2201_11133_amd import synth
    print("case: tiny member 64 windows", flush=True)
    blob = synth.tiny_weights(0)
    x, injs = synth.make_windows(100, 64, 8)
    a, p = oracle_params(blob, "tiny")
    z64 = forward_window(a, p, x.astype(np.float64))                    # [64, 4096]
    m = g.Model(g.tiny_arch(), blob, "fp32")
    dev = [to_dev(x[i]) for i in range(64)]                               # 64 streams of one window each
    z2 = m.forward(dev, 4096, 256, out_mode=2).cpu().numpy().reshape(64, 4096)
    e0 = m.forward(dev, 4096, 256, out_mode=0)
    torch.cuda.synchronize()
    dp = np.abs(sigmoid64(z2) - sigmoid64(z64)).max()
    print(f"tiny max|dp| = {dp:.3g}", flush=True)
    assert dp <= FP32_P_TOL
    assert np.array_equal(e0.cpu().numpy(), z2.reshape(-1))              # one member, one window per stream
    offs = np.arange(65) * 4096
    got = g.triggers(e0, offs, 0.9, 4096)
    assert len(got) <= 64
    # the trigger list of the oracle's own FP64 scores, fragile decisions exempt
    _check_triggers_against_oracle(g, e0, z64.reshape(-1), offs, "tiny member")
    m.close()


# ---------------------------------------------------------------- layer-local parity
@pytest.mark.parametrize("layer", [0, 5, 9, 19, 29])
def test_layer_parity_fp32(g, full_model, full_blob, layer):
    """One gated layer on the GPU vs the oracle layer applied to the same input bits, bounded by the
    forward error of a length-K dot product, |d| <= K u (|W| |x|) (Higham, Accuracy and Stability of
    Numerical Algorithms, sec. 3.1)."""
    from oracle.forward import gated_layer, shift_right
    print(f"case: layer {layer}", flush=True)
    a, p = oracle_params(full_blob)
    T, nw, C = 1024, 2, 128
    rng = np.random.default_rng(layer)
    x = (rng.standard_normal((nw, T, C)) * 3).astype(np.float32)
    sk = (rng.standard_normal((nw, T, C)) * 4).astype(np.float32)
    x_d, sk_d = to_dev(x), to_dev(sk.copy())
    pre_d = torch.empty((nw, T, 2 * C), dtype=torch.float32, device="cuda")
    xo_d = torch.zeros((nw, T, C), dtype=torch.float32, device="cuda")
    full_model.debug_layer(0, layer, x_d, nw, T, pre_d, xo_d, sk_d)
    torch.cuda.synchronize()
    skip_in = np.zeros_like(sk, dtype=np.float64) if layer == 0 else sk.astype(np.float64)
    pre, gg, xo, sko = gated_layer(a, p, layer, x.astype(np.float64), skip_in)
    d = a.dilation(layer)
    W = p[f"dil{layer}.W"]
    ax = np.concatenate([np.abs(shift_right(x.astype(np.float64), d)), np.abs(x)], axis=-1)
    aW = np.concatenate([np.abs(W[:, :, 0]).T, np.abs(W[:, :, 1]).T], axis=0)
    bound = 256 * U32 * (ax @ aW) + U32 * np.abs(pre) + 1e-30
    pre_g = pre_d.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(pre_g - pre) <= bound), np.max(np.abs(pre_g - pre) / bound)
    # gate error: derivative magnitude <= 1 times the pre-activation error, plus a few ulp
    dg = np.max(np.abs(pre_g - pre)) + 8 * U32
    Ws = p[f"skip{layer}.W"]
    sk_bound = 128 * U32 * (np.abs(gg) @ np.abs(Ws).T) + np.abs(Ws).sum(axis=1) * dg + 2 * U32 * (np.abs(sko) + 1)
    assert np.all(np.abs(sk_d.cpu().numpy() - sko) <= sk_bound)
    if layer < a.n_layers - 1:
        Wr = p[f"res{layer}.W"]
        xo_bound = 128 * U32 * (np.abs(gg) @ np.abs(Wr).T) + np.abs(Wr).sum(axis=1) * dg + 2 * U32 * (np.abs(xo) + 1)
        assert np.all(np.abs(xo_d.cpu().numpy() - xo) <= xo_bound)


# ---------------------------------------------------------------- full member end to end
def test_full_member_windows_ragged_tail(g, full_model, full_blob):
    """Per-window logits of a short stream: 8 windows, last one ragged (zero-filled past the end)."""
    from oracle.forward import forward_window
    from oracle.stream import gather_windows, stitch
    from paper_2201_11133_amd import synth
    print("case: full member ragged stream", flush=True)
    W, S = 4096, 256
    L = W + 6 * S + 100
    x, _ = synth.make_stream(105, L / 4096, 0)
    a, p = oracle_params(full_blob)
    zw64 = forward_window(a, p, gather_windows(x.astype(np.float64), W, S))   # [8, W]
    xd = to_dev(x)
    z2 = full_model.forward([xd], W, S, out_mode=2).cpu().numpy().reshape(-1, W)
    e0 = full_model.forward([xd], W, S, out_mode=0).cpu().numpy()
    assert z2.shape == zw64.shape == (8, W)
    dp = np.abs(sigmoid64(z2) - sigmoid64(zw64)).max()
    print(f"full fp32 per-window max|dp| = {dp:.3g}", flush=True)
    assert dp <= FP32_P_TOL
    # stitched output is exactly the owner-window selection of the per-window output
    assert np.array_equal(e0, stitch(z2, L, W, S).astype(np.float32))


def test_output_modes_and_multi_stream(g, full_model, full_blob):
    """Several streams (one empty, one shorter than a window) in one call; mode 1 layout."""
    from oracle.forward import forward_stream
    from paper_2201_11133_amd import synth
    print("case: multi-stream modes", flush=True)
    W, S = 4096, 256
    lens = [5000, 0, 3000, 4096]
    xs = [synth.make_stream(200 + i, max(n, 1) / 4096, 0)[0][:n] for i, n in enumerate(lens)]
    devs = [to_dev(x) if len(x) else torch.zeros((0, 2), dtype=torch.float32, device="cuda") for x in xs]
    m2 = g.Model(g.full_arch(), np.stack([full_blob, full_blob]), "fp32")
    out1 = m2.forward(devs, W, S, out_mode=1).cpu().numpy()
    N = sum(lens)
    e, per = out1[:N], out1[N:].reshape(2, N)
    assert np.array_equal(per[0], per[1]) and np.array_equal(e, per[0])     # identical members: e = z
    a, p = oracle_params(full_blob)
    off = 0
    for x, n in zip(xs, lens):
        if n:
            z64 = forward_stream(a, p, x.astype(np.float64))
            assert np.abs(sigmoid64(e[off:off + n]) - sigmoid64(z64)).max() <= FP32_P_TOL
        off += n
    m2.close()


def test_parity_slice_16s(g, full_model, full_blob):
    """A 16 s stream (241 windows, one chirp), stitched, vs the oracle's streaming pass (equal to the
    owner-window stitch because RF - 1 <= W - S)."""
    from oracle.forward import forward_stream
    from paper_2201_11133_amd import synth
    print("case: 16 s parity slice", flush=True)
    x, _ = synth.make_stream(101, 16.0, 1, spacing=10.0, margin=4.0)
    xd = to_dev(x)
    e = full_model.forward([xd], 4096, 256, out_mode=0).cpu().numpy()
    a, p = oracle_params(full_blob)
    z64 = forward_stream(a, p, x.astype(np.float64))
    dp = np.abs(sigmoid64(e) - sigmoid64(z64))
    print(f"16 s slice max|dp| = {dp.max():.3g}, p99 = {np.quantile(dp, 0.99):.3g}", flush=True)
    assert dp.max() <= FP32_P_TOL


def test_full_size_stream_sampled_parity(g, full_model, full_blob):
    """The single-member FP32 workload at its full size: 4096 s of two-channel strain (16,777,216
    samples, 65,521 windows, 20 chirps), one forward in the batching the benchmark uses. Sampled
    windows (the first, a middle one, one around each of three injections, the last two, whose tail
    is zero-filled) are recomputed by the oracle window by window; every sample they own must match
    within the FP32 tolerance."""
    from oracle.forward import forward_window
    from oracle.stream import gather_windows, n_windows, owner
    from paper_2201_11133_amd import synth
    print("case: full-size 4096 s stream, sampled windows", flush=True)
    W, S = 4096, 256
    x, injs = synth.make_stream(101, 4096.0, 20, spacing=10.0, margin=4.0)
    L = x.shape[0]
    nw = n_windows(L, W, S)
    assert nw == 65521
    e = full_model.forward([to_dev(x)], W, S, out_mode=0).cpu().numpy()
    a, p = oracle_params(full_blob)
    picks = {0, nw // 2, nw - 2, nw - 1}
    for inj in injs[:3]:
        picks.add(int(owner(np.array([int(inj.tc * 4096)]), W, S)[0][0]))
    k_of, pos_of = owner(np.arange(L), W, S)
    worst = 0.0
    for k in sorted(picks):
        z64 = forward_window(a, p, gather_windows(x[k * S: k * S + W + S].astype(np.float64), W, S)[:1])[0]
        rows = np.nonzero(k_of == k)[0]
        dp = np.abs(sigmoid64(e[rows]) - sigmoid64(z64[pos_of[rows]]))
        worst = max(worst, float(dp.max()))
    print(f"full-size sampled windows {sorted(picks)}: max|dp| = {worst:.3g}", flush=True)
    assert worst <= FP32_P_TOL


def test_arg_errors_on_device(g, full_model):
    xd = torch.zeros((5000, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(g.GwdError) as ei:
        full_model.forward([xd], 4096, 2000, out_mode=0)    # W - S < RF - 1
    assert ei.value.code == g.ERR_SHAPE
    with pytest.raises(g.GwdError) as ei:
        full_model.forward([xd], 3008, 256, out_mode=0)     # W < RF
    assert ei.value.code == g.ERR_SHAPE
    out = torch.empty(10, dtype=torch.float32, device="cuda")
    with pytest.raises(g.GwdError) as ei:
        full_model.forward([xd], 4096, 256, out_mode=0, out=out)
    assert ei.value.code == g.ERR_CAPACITY


# ---------------------------------------------------------------- FP32 trigger lists vs the FP64 oracle's
TRIG_MARGIN = 1e-4   # logit distance within which a trigger decision counts as fragile


def _oracle_scores(blobs, x):
    """Ensemble logit of the FP64 oracle (one causal pass per member, members in parallel threads)."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle.forward import forward_stream
    from oracle.stream import ensemble
    a, _ = oracle_params(blobs[0])
    x64 = x.astype(np.float64)
    from oracle.arch import unpack
    with ThreadPoolExecutor(max_workers=len(blobs)) as ex:
        zs = list(ex.map(lambda b: forward_stream(a, unpack(a, b.astype(np.float64)), x64), blobs))
    return ensemble(zs)


def _check_triggers_against_oracle(g, e_dev, e64, offs, label):
    """GPU trigger list (FP32 scores) == the oracle rule on the FP64 oracle's scores, except for
    decisions that are fragile in the oracle's scores. If every score differs by less than half the
    margin, a decision can only flip where the oracle's score lies within the margin of the
    threshold or of its strongest in-window competitor: exactly the fragile set."""
    from oracle.triggers import triggers as otrig
    from tests.gpu_common import fragile_keys
    e = e_dev.cpu().numpy().astype(np.float64)
    dz = float(np.max(np.abs(e - e64)))
    got = {(int(s), int(a)) for s, a, _, _ in g.triggers(e_dev, offs, 0.9, 4096)}
    ref = {(int(s), int(a)) for s, a, _, _ in otrig(e64, offs, 0.9, 4096)}
    fragile = fragile_keys(e64, offs, 0.9, 4096, TRIG_MARGIN)
    diff = got ^ ref
    print(f"{label}: oracle {len(ref)} triggers, gpu {len(got)}, max|dz| = {dz:.3g}, "
          f"fragile decisions {len(fragile)}, differing {len(diff)} (all fragile: {diff <= fragile})", flush=True)
    assert dz < TRIG_MARGIN / 2, dz
    assert diff <= fragile, sorted(diff - fragile)
    return got, ref


@pytest.mark.timeout(900)
def test_fp32_triggers_match_oracle_64s_slice(g, full_model, full_blob):
    """The single-member FP32 workload's parity slice: the first 64 s (1,009 windows) of the 4096 s
    stream with 20 chirps, stitched and clustered on the device, against the trigger list of the
    oracle's FP64 scores."""
    from paper_2201_11133_amd import synth
    print("case: fp32 triggers, 64 s slice of the 4096 s stream", flush=True)
    x, _ = synth.make_stream(101, 4096.0, 20, spacing=10.0, margin=4.0)
    x = np.ascontiguousarray(x[:64 * 4096])
    e_dev = full_model.forward([to_dev(x)], 4096, 256, out_mode=0)
    e64 = _oracle_scores([full_blob], x)
    _check_triggers_against_oracle(g, e_dev, e64, [0, len(x)], "64 s slice")


@pytest.mark.timeout(900)
def test_fp32_triggers_match_oracle_injections(g, full_model, full_blob):
    """16 s around each of the first two injections of the 4096 s stream (chirp near the middle),
    scored as two streams in one call."""
    from paper_2201_11133_amd import synth
    print("case: fp32 triggers, slices around two injections", flush=True)
    x, injs = synth.make_stream(101, 4096.0, 20, spacing=10.0, margin=4.0)
    parts = []
    for inj in injs[:2]:
        a0 = int(inj.tc * 4096) - 8 * 4096
        parts.append(np.ascontiguousarray(x[a0:a0 + 16 * 4096]))
    e_dev = full_model.forward([to_dev(p) for p in parts], 4096, 256, out_mode=0)
    e64 = np.concatenate([_oracle_scores([full_blob], p) for p in parts])
    offs = [0, len(parts[0]), len(parts[0]) + len(parts[1])]
    _check_triggers_against_oracle(g, e_dev, e64, offs, "injection slices")


@pytest.mark.timeout(900)
def test_fp32_ensemble_triggers_match_oracle(g):
    """A 4-member FP32 ensemble (member seeds 11-14) over 16 s with two chirps: the ensemble minimum
    and the triggers on the device against the oracle's."""
    from paper_2201_11133_amd import synth
    print("case: fp32 4-member ensemble triggers, 16 s", flush=True)
    blobs = np.stack([synth.full_weights(11 + i) for i in range(4)])
    x, _ = synth.make_stream(106, 16.0, 2)
    m = g.Model(g.full_arch(), blobs, "fp32")
    e_dev = m.forward([to_dev(x)], 4096, 256, out_mode=0)
    torch.cuda.synchronize()
    e64 = _oracle_scores(list(blobs), x)
    m.close()
    dp = np.abs(sigmoid64(e_dev.cpu().numpy()) - sigmoid64(e64)).max()
    print(f"4-member fp32 ensemble: max|dp| = {dp:.3g}", flush=True)
    assert dp <= FP32_P_TOL
    _check_triggers_against_oracle(g, e_dev, e64, [0, len(x)], "4-member ensemble")
