"""Pins for the trigger rule: brute force, closed-form streams, spacing, stream isolation."""
import math

import numpy as np
import pytest

from oracle.triggers import logit_threshold, triggers, triggers_brute

LN9 = 2.1972245773362196


def keys(recs):
    return [(s, a) for s, a, _, _ in recs]


def test_threshold_is_ln9():
    assert logit_threshold(0.9) == math.log(9.0)
    assert abs(logit_threshold(0.9) - LN9) < 1e-15


@pytest.mark.parametrize("seed", range(12))
def test_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    wc = int(rng.integers(1, 40))
    e = rng.standard_normal(n) * 3 + 1
    if seed % 3 == 0:
        e = np.round(e)          # many exact ties
    cuts = np.sort(rng.choice(np.arange(1, n), size=min(3, n - 1), replace=False)) if n > 3 else []
    offs = [0] + [int(c) for c in cuts] + [n]
    assert keys(triggers(e, offs, 0.9, wc)) == triggers_brute(e, offs, 0.9, wc)


def test_constant_stream_triggers_at_first_sample():
    e = np.full(10000, 3.0)
    assert keys(triggers(e, [0, 10000])) == [(0, 0)]
    e = np.full(10000, 1.0)   # below ln 9
    assert triggers(e, [0, 10000]) == []


def test_increasing_stream_triggers_at_last_sample():
    e = np.linspace(2.5, 9.0, 7000)
    assert keys(triggers(e, [0, 7000])) == [(0, 6999)]


def test_threshold_inclusive():
    e = np.full(5, -5.0)
    e[2] = LN9
    assert keys(triggers(e, [0, 5], 0.9, 4)) == [(0, 2)]
    e[2] = np.nextafter(LN9, -np.inf)
    assert triggers(e, [0, 5], 0.9, 4) == []


def test_ties_go_to_earliest():
    e = np.zeros(30)
    e[[5, 9]] = 4.0
    assert keys(triggers(e, [0, 30], 0.9, 4)) == [(0, 5)]
    assert keys(triggers(e, [0, 30], 0.9, 3)) == [(0, 5), (0, 9)]


def test_spacing_invariant():
    rng = np.random.default_rng(99)
    e = rng.standard_normal(200000) * 4
    wc = 4096
    a = np.array([x for _, x, _, _ in triggers(e, [0, e.size], 0.9, wc)])
    assert a.size > 5
    assert np.all(np.diff(a) >= wc + 1)


def test_streams_are_isolated():
    """A large value in stream 0 must not suppress a peak at the start of stream 1."""
    e = np.zeros(40)
    e[19] = 10.0      # last sample of stream 0
    e[20] = 3.0       # first sample of stream 1
    assert keys(triggers(e, [0, 20, 40], 0.9, 8)) == [(0, 19), (1, 0)]


def test_records_carry_logit_and_probability():
    e = np.zeros(10)
    e[4] = 3.0
    (s, a, z, p), = triggers(e, [0, 10], 0.9, 4)
    assert (s, a, z) == (0, 4, 3.0) and abs(p - 1 / (1 + math.exp(-3.0))) < 1e-15


def test_empty_streams():
    assert triggers(np.zeros(0), [0, 0, 0]) == []


def _fragile_brute(e, offsets, p_thr, wc, margin):
    import math
    thr = math.log(p_thr / (1 - p_thr))
    out = set()
    for s in range(len(offsets) - 1):
        seg = [float(v) for v in e[offsets[s]:offsets[s + 1]]]
        n = len(seg)
        for a in range(n):
            nb = [seg[b] for b in range(max(0, a - wc), min(n, a + wc + 1)) if b != a]
            comp = max(nb) if nb else -math.inf
            if abs(seg[a] - thr) < margin or abs(seg[a] - comp) < margin:
                out.add((s, a))
    return out


@pytest.mark.parametrize("seed", range(4))
def test_fragile_decisions_brute_force(seed):
    """The fragile set against its definition, loop by loop, on quantised streams (many near ties)."""
    from oracle.triggers import fragile_decisions
    rng = np.random.default_rng(seed)
    lens = [0, 1, 37, 200, 5]
    e = np.round(rng.normal(2.2, 0.5, sum(lens)) * 200) / 200
    offs = np.concatenate([[0], np.cumsum(lens)])
    for wc, m in [(1, 1e-3), (7, 6e-3), (50, 2e-2)]:
        assert fragile_decisions(e, offs, 0.9, wc, m) == _fragile_brute(e, offs, 0.9, wc, m)


@pytest.mark.parametrize("seed", range(6))
def test_small_perturbations_flip_only_fragile_decisions(seed):
    """Scores perturbed by less than margin / 2 give a trigger list that differs from the
    unperturbed one only at fragile decisions (the property the FP32 parity tests rely on)."""
    from oracle.triggers import fragile_decisions
    rng = np.random.default_rng(seed)
    lens = [300, 1, 450]
    offs = np.concatenate([[0], np.cumsum(lens)])
    e = np.round(rng.normal(2.2, 0.3, sum(lens)) * 100) / 100
    margin = 0.02
    ref = set(triggers_brute(e, offs, 0.9, 20))
    fr = fragile_decisions(e, offs, 0.9, 20, margin)
    for _ in range(20):
        ep = e + rng.uniform(-0.49, 0.49, e.size) * margin
        got = set(triggers_brute(ep, offs, 0.9, 20))
        assert (got ^ ref) <= fr
