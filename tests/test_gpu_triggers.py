"""GPU trigger kernel (through the C ABI) vs the oracle rule on the same scores: bit-exact lists."""
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


def ref(e, offs, p=0.9, wc=4096):
    from oracle.triggers import triggers
    return [(s, a) for s, a, _, _ in triggers(e.astype(np.float64), offs, p, wc)]


def got(g, e, offs, p=0.9, wc=4096, capacity=None):
    return [(s, a) for s, a, _, _ in g.triggers(to_dev(e), offs, p, wc, capacity)]


@pytest.mark.parametrize("wc", [1, 7, 64, 4096, 65536])
@pytest.mark.parametrize("seed", [0, 1])
def test_random_multistream(g, wc, seed):
    print(f"case: triggers random wc={wc} seed={seed}", flush=True)
    rng = np.random.default_rng(seed)
    lens = [0, 1, 5, wc, wc + 1, 3 * wc + 17, 200000, 0, 12345]
    e = (rng.standard_normal(sum(lens)) * 3).astype(np.float32)
    if seed == 1:
        e = np.round(e).astype(np.float32)   # many exact ties
    offs = np.concatenate([[0], np.cumsum(lens)])
    assert got(g, e, offs, 0.9, wc) == ref(e, offs, 0.9, wc)


def test_large_stream(g):
    print("case: triggers 20M samples", flush=True)
    rng = np.random.default_rng(5)
    e = (rng.standard_normal(20_000_000) * 4).astype(np.float32)
    offs = np.array([0, e.size])
    r = ref(e, offs)
    assert got(g, e, offs) == r and len(r) > 1000


def test_closed_forms(g):
    offs = np.array([0, 10000, 17000, 17005])
    e = np.concatenate([np.full(10000, 3.0), np.linspace(2.5, 9.0, 7000), np.full(5, 1.0)]).astype(np.float32)
    assert got(g, e, offs) == [(0, 0), (1, 6999)]


def test_records_and_threshold_edge(g):
    e = np.full(100, -5.0, dtype=np.float32)
    ln9 = np.float32(np.log(9.0))
    # the float32 value just above ln 9 passes, the one just below does not
    e[10] = np.nextafter(ln9, np.float32(10)) if float(ln9) < np.log(9.0) else ln9
    e[60] = np.nextafter(e[10], np.float32(-10))
    recs = g.triggers(to_dev(e), [0, 100], 0.9, 4)
    assert [(s, a) for s, a, _, _ in recs] == [(0, 10)]
    s, a, z, p = recs[0]
    assert z == e[10] and abs(p - 1 / (1 + np.exp(-float(z)))) < 1e-7


def test_capacity_overflow(g):
    e = np.zeros(10 * 4097, dtype=np.float32)
    e[::4097] = 5.0
    offs = np.array([0, e.size])
    with pytest.raises(g.GwdError) as ei:
        g.triggers(to_dev(e), offs, 0.9, 4096, capacity=3)
    assert ei.value.code == g.ERR_CAPACITY


def test_nonfinite(g):
    e = np.zeros(9000, dtype=np.float32)
    e[4500] = np.nan
    with pytest.raises(g.GwdError) as ei:
        g.triggers(to_dev(e), [0, 9000], 0.9, 4096)
    assert ei.value.code == g.ERR_NONFINITE
    e[4500] = np.inf
    with pytest.raises(g.GwdError) as ei:
        g.triggers(to_dev(e), [0, 9000], 0.9, 4096)
    assert ei.value.code == g.ERR_NONFINITE
