"""Time-slide background on the GPU: slid copies against the oracle (bit-exact moves), the forward and
the triggers of slid streams against those of the same streams slid by the oracle on the host, and the
false-alarm counts of the background triggers against the oracle's."""
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


@pytest.mark.parametrize("L", [1, 5, 4097, 100003])
def test_slides_match_oracle(g, L):
    from oracle.background import time_slide
    print(f"case: slides L={L}", flush=True)
    x = np.random.default_rng(L).standard_normal((L, 2)).astype(np.float32)
    shifts = [0, 1, L - 1, L, -3, 2 * L + 5, 10 ** 12 + 7, -(10 ** 12) - 11]
    xd = to_dev(x)
    got = g.time_slide(xd, shifts).cpu().numpy()
    for k, s in enumerate(shifts):
        assert np.array_equal(got[k], time_slide(x, s)), s
    # planar source (two separate channel buffers): the same copies
    c0, c1 = to_dev(x[:, 0].copy()), to_dev(x[:, 1].copy())
    got2 = g.time_slide((c0, c1), shifts).cpu().numpy()
    assert np.array_equal(got2, got)


def test_empty_stream(g):
    x = torch.zeros((0, 2), dtype=torch.float32, device="cuda")
    out = g.time_slide(x, [3, 4])
    assert tuple(out.shape) == (2, 0, 2)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_background_forward_and_far(g, prec):
    """K slides of one stream in one forward call: the ensemble scores and triggers equal those of the
    same slides made on the host by the oracle and uploaded; the false-alarm counts of the triggers
    equal the oracle's count."""
    from oracle.background import far_curve, time_slide
    from paper_2201_11133_amd import synth
    print(f"case: background {prec}", flush=True)
    x, _ = synth.make_stream(410, 12.0, 2)
    L = x.shape[0]
    shifts = [8 * 4096, 8 * 4096 * 2 + 17, L - 4096]
    blobs = np.stack([synth.full_weights(11 + i) for i in range(2)])
    m = g.Model(g.full_arch(), blobs, prec)
    slid = g.time_slide(to_dev(x), shifts)
    dev_streams = [slid[k] for k in range(len(shifts))]
    host_streams = [to_dev(time_slide(x, s)) for s in shifts]
    a = m.forward(dev_streams, 4096, 256, 0).clone()
    b = m.forward(host_streams, 4096, 256, 0).clone()
    assert torch.equal(a, b)
    offs = [k * L for k in range(len(shifts) + 1)]
    ta = g.triggers(a, offs)
    tb = g.triggers(b, offs)
    assert ta == tb
    thr = [np.log(9.0), 3.0, 5.0, 8.0]
    live = len(shifts) * L / 4096.0
    counts, far = g.far_curve(ta, thr, live)
    c_o, f_o = far_curve([z for _, _, z, _ in ta], thr, live)
    assert np.array_equal(counts, c_o) and np.array_equal(far, f_o)
    assert counts[0] == len(ta)
    m.close()
