"""The allocation-free trigger entry point (gwd_triggers_noalloc, static device scratch) through the
C ABI: its records equal those of gwd_triggers, bit for bit, on two calls in a row, the second on a
smaller input, so that the array's contents from the first call must not leak into the second."""
import ctypes

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


def call(g, fn, e, offs, p, wc, cap):
    offs = np.ascontiguousarray(np.asarray(offs, np.int64))
    buf = (g.Trigger * max(cap, 1))()
    nf = ctypes.c_int64(-1)
    code = fn(g._ptr(e), offs.ctypes.data, offs.size - 1, p, wc, buf, cap, ctypes.byref(nf), None)
    recs = [(buf[i].stream, buf[i].sample, buf[i].logit, buf[i].prob) for i in range(min(max(nf.value, 0), cap))]
    return code, nf.value, recs


def scores(seed, lens, ties):
    rng = np.random.default_rng(seed)
    e = (rng.standard_normal(int(sum(lens))) * 3).astype(np.float32)
    if ties:
        e = np.round(e).astype(np.float32)
    return e, np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


def test_noalloc_matches_allocating_entry_twice(g):
    from oracle.triggers import triggers as otrig
    cases = [  # (seed, stream lengths, ties, cluster window): the second call is smaller
        (5, [0, 1, 4097, 1_000_003, 200_000, 12_345], False, 4096),
        (6, [50_000, 3, 9_999], True, 64),
    ]
    for seed, lens, ties, wc in cases:
        print(f"case: noalloc triggers seed={seed} lens={lens} wc={wc}", flush=True)
        e_h, offs = scores(seed, lens, ties)
        e = to_dev(e_h)
        n_tiles = int(sum(-(-L // wc) for L in lens))
        need = g.lib.gwd_triggers_noalloc_scratch_bytes(offs.ctypes.data, len(lens), wc)
        assert 0 < need <= 16 << 20
        c0, n0, r0 = call(g, g.lib.gwd_triggers, e, offs, 0.9, wc, n_tiles)
        c1, n1, r1 = call(g, g.lib.gwd_triggers_noalloc, e, offs, 0.9, wc, n_tiles)
        torch.cuda.synchronize()
        assert c0 == g.OK and c1 == g.OK, (c0, c1, g.last_error())
        assert n1 == n0 and n0 > 0
        assert r1 == r0
        # and the list is the oracle rule's on the same scores
        assert [(s, a) for s, a, _, _ in r1] == [(s, a) for s, a, _, _ in otrig(e_h.astype(np.float64), offs, 0.9, wc)]
        # capacity overflow behaves the same: the first records, the true count, GWD_ERR_CAPACITY
        c2, n2, r2 = call(g, g.lib.gwd_triggers_noalloc, e, offs, 0.9, wc, 2)
        assert c2 == g.ERR_CAPACITY and n2 == n0 and r2 == r0[:2]


def test_noalloc_nonfinite_then_clean(g):
    print("case: noalloc non-finite score, then a clean call", flush=True)
    e_h, offs = scores(7, [9000, 9000], False)
    bad = e_h.copy()
    bad[12000] = np.nan
    c, n, _ = call(g, g.lib.gwd_triggers_noalloc, to_dev(bad), offs, 0.9, 4096, 8)
    assert c == g.ERR_NONFINITE and n == 0
    # the flag left in the array by the call above must not reach the next one
    c0, n0, r0 = call(g, g.lib.gwd_triggers, to_dev(e_h), offs, 0.9, 4096, 8)
    c1, n1, r1 = call(g, g.lib.gwd_triggers_noalloc, to_dev(e_h), offs, 0.9, 4096, 8)
    assert (c0, n0) == (c1, n1) == (g.OK, n0) and r1 == r0
