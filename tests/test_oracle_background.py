"""Pins for the time-slide background oracle: index definition by brute force, group structure of
circular shifts, channel 0 untouched, the destroyed coincidence, and false-alarm counting."""
import numpy as np
import pytest

from oracle.background import far_curve, time_slide
from oracle.triggers import triggers


def rand_stream(seed, L):
    return np.random.default_rng(seed).standard_normal((L, 2))


@pytest.mark.parametrize("L,shift", [(1, 0), (1, 5), (7, 3), (7, -2), (7, 7), (7, 23), (50, 49), (50, -51)])
def test_index_definition_brute_force(L, shift):
    x = rand_stream(L + 100, L)
    y = time_slide(x, shift)
    for t in range(L):
        assert y[t, 0] == x[t, 0]
        # the index written out without modular arithmetic
        u = t + shift
        while u >= L:
            u -= L
        while u < 0:
            u += L
        assert y[t, 1] == x[u, 1]


def test_identity_and_group_structure():
    x = rand_stream(1, 97)
    assert np.array_equal(time_slide(x, 0), x)
    assert np.array_equal(time_slide(x, 97), x)
    assert np.array_equal(time_slide(x, -97 * 3), x)
    # composing two slides adds their shifts; a slide is undone by its negative
    assert np.array_equal(time_slide(time_slide(x, 30), 50), time_slide(x, 80))
    assert np.array_equal(time_slide(time_slide(x, 41), -41), x)
    # a slide permutes channel 1: same multiset of values, channel 0 untouched
    y = time_slide(x, 13)
    assert np.array_equal(np.sort(y[:, 1]), np.sort(x[:, 1]))
    assert np.array_equal(y[:, 0], x[:, 0])


def test_empty_stream():
    x = np.zeros((0, 2))
    assert time_slide(x, 5).shape == (0, 2)


def test_coincidence_is_destroyed():
    """A burst present in both channels at the same time is no longer coincident after a slide
    longer than the burst: the sample-wise product of the channels loses its peak."""
    L, a, w = 4000, 1500, 40
    x = np.zeros((L, 2))
    x[a:a + w, :] = 1.0
    assert np.sum(x[:, 0] * x[:, 1]) == w
    y = time_slide(x, 1000)
    assert np.sum(y[:, 0] * y[:, 1]) == 0.0
    # the slid channel carries the burst 1000 samples earlier
    assert np.array_equal(np.nonzero(y[:, 1])[0], np.arange(a - 1000, a - 1000 + w))


def test_far_counts_brute_force_and_monotone():
    rng = np.random.default_rng(3)
    z = rng.normal(3.0, 2.0, 500)
    thr = np.linspace(-1.0, 9.0, 41)
    counts, rate = far_curve(z, thr, 3600.0)
    for i, t in enumerate(thr):
        assert counts[i] == sum(1 for v in z if v >= t)
    assert np.all(np.diff(counts) <= 0)
    assert np.allclose(rate, counts / 3600.0)
    # inclusive comparison
    c, _ = far_curve([1.0, 2.0, 2.0, 3.0], [2.0], 1.0)
    assert c[0] == 3


def test_far_curve_from_one_low_threshold_list():
    """Clustering does not involve the threshold: the triggers at a higher threshold are exactly the
    records of the low-threshold list whose score reaches it."""
    rng = np.random.default_rng(9)
    e = np.cumsum(rng.standard_normal(20000)) * 0.05 + rng.standard_normal(20000)
    low = triggers(e, [0, e.size], 0.6, 300)
    for p in (0.7, 0.9, 0.97):
        hi = triggers(e, [0, e.size], p, 300)
        zt = np.log(p / (1 - p))
        assert [(s, a) for s, a, _, _ in hi] == [(s, a) for s, a, z, _ in low if z >= zt]
        counts, _ = far_curve([z for _, _, z, _ in low], [zt], 1.0)
        assert counts[0] == len(hi)
