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
