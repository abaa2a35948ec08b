"""The paper's post-processing on the GPU: peak finding against SciPy's find_peaks (the oracle) on
seeded signals made on the host, bit for bit in peak indices and widths; float64 probabilities;
edge cases."""
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


def signal(kind, n, rng):
    if kind == "noise":
        return rng.standard_normal(n)
    if kind == "plateaus":
        return np.round(rng.standard_normal(n) * 2) / 2
    if kind == "walk":
        return np.cumsum(rng.standard_normal(n))
    if kind == "prob":   # model-like probabilities: smooth logits, saturated stretches
        z = np.convolve(rng.standard_normal(n + 400) * 8, np.ones(400) / 20, mode="valid")[:n]
        return 1 / (1 + np.exp(-z))
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["noise", "plateaus", "walk", "prob"])
@pytest.mark.parametrize("n", [3, 37, 5000, 300001])
def test_find_peaks_matches_scipy(g, kind, n):
    from oracle.postproc import find_peaks
    print(f"case: find_peaks {kind} n={n}", flush=True)
    rng = np.random.default_rng(n + len(kind))
    x = signal(kind, n, rng)
    for height, wmin in [(float(np.quantile(x, 0.5)), 0.0), (float(np.quantile(x, 0.9)), 3.0), (-1e300, 2048.0)]:
        p, w = g.find_peaks(to_dev(x), height, wmin)
        rp, rw = find_peaks(x, height, wmin)
        assert np.array_equal(p, rp), (height, wmin)
        assert np.array_equal(w, rw), (height, wmin)


def test_edge_cases(g):
    from oracle.postproc import find_peaks
    for x in [np.zeros(0), np.zeros(1), np.array([1.0, 2.0]), np.ones(100), np.arange(100.0),
              np.array([0, 1, 3, 3, 3, 3, 1, 0, 5, 5, 0, 2.0]), np.array([5.0, 1, 5]), np.array([1.0, 2, 2])]:
        xd = to_dev(x) if x.size else torch.zeros(0, dtype=torch.float64, device="cuda")
        p, w = g.find_peaks(xd, -1.0, 0.0)
        rp, rw = find_peaks(x, -1.0, 0.0) if x.size else (np.zeros(0, np.int64), np.zeros(0))
        assert np.array_equal(p, rp) and np.array_equal(w, rw)


def test_nonfinite_and_capacity(g):
    x = np.random.default_rng(1).standard_normal(1000)
    x[500] = np.nan
    with pytest.raises(g.GwdError) as ei:
        g.find_peaks(to_dev(x), 0.0, 0.0)
    assert ei.value.code == g.ERR_NONFINITE
    x[500] = 0.0
    p, _ = g.find_peaks(to_dev(x), 0.0, 0.0)
    assert p.size > 3
    with pytest.raises(g.GwdError) as ei:
        g.find_peaks(to_dev(x), 0.0, 0.0, capacity=3)
    assert ei.value.code == g.ERR_CAPACITY


def test_prob64(g):
    """float64 probabilities from float32 logits: within 4 ulp of NumPy (both round exp to within 1 ulp)."""
    z = (np.random.default_rng(2).standard_normal(100000) * 20).astype(np.float32)
    p = g.prob64(to_dev(z)).cpu().numpy()
    ref = 1.0 / (1.0 + np.exp(-z.astype(np.float64)))
    assert np.all(np.abs(p - ref) <= 4 * np.spacing(ref))
