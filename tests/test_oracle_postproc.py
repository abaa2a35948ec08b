"""Pins for the post-processing oracle: the peak definition written out by brute force (local maxima with
plateaus, prominence bases, half-prominence width with interpolation), closed-form shapes, and the
coincidence rule by brute force."""
import numpy as np
import pytest

from oracle.postproc import coincident_events, find_peaks


def brute_peaks(x, height, min_width):
    """The definition, sample by sample, in plain Python."""
    n = len(x)
    out, widths = [], []
    for i in range(1, n - 1):
        if not x[i - 1] < x[i]:
            continue
        j = i + 1
        while j < n - 1 and x[j] == x[i]:
            j += 1
        if not x[j] < x[i]:
            continue
        p = (i + j - 1) // 2
        if x[p] < height:
            continue
        # bases: lowest points before a strictly higher sample on each side
        lmin, lb, k = x[p], p, p
        while k >= 0 and x[k] <= x[p]:
            if x[k] < lmin:
                lmin, lb = x[k], k
            k -= 1
        rmin, rb, k = x[p], p, p
        while k <= n - 1 and x[k] <= x[p]:
            if x[k] < rmin:
                rmin, rb = x[k], k
            k += 1
        level = x[p] - (x[p] - max(lmin, rmin)) * 0.5
        k = p
        while lb < k and level < x[k]:
            k -= 1
        left = float(k) + ((level - x[k]) / (x[k + 1] - x[k]) if x[k] < level else 0.0)
        k = p
        while k < rb and level < x[k]:
            k += 1
        right = float(k) - ((level - x[k]) / (x[k - 1] - x[k]) if x[k] < level else 0.0)
        if right - left >= min_width:
            out.append(p)
            widths.append(right - left)
    return np.array(out, dtype=np.int64), np.array(widths)


@pytest.mark.parametrize("seed", range(24))
def test_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    kind = seed % 4
    if kind == 0:
        x = rng.standard_normal(n)
    elif kind == 1:
        x = np.round(rng.standard_normal(n) * 2) / 2          # plateaus and ties
    elif kind == 2:
        x = np.cumsum(rng.standard_normal(n))                  # long slopes
    else:
        x = 1 / (1 + np.exp(-np.clip(rng.standard_normal(n) * 30, -60, 60)))  # saturated probabilities
    h = float(np.quantile(x, 0.3))
    w = float(rng.uniform(0, 6))
    p, wd = find_peaks(x, h, w)
    bp, bw = brute_peaks(x, h, w)
    assert np.array_equal(p, bp)
    assert np.array_equal(wd, bw)


def test_triangle_closed_form():
    """A triangle of height 1 and half-base 100 on zeros: prominence 1, width at half height = 100."""
    x = np.zeros(1001)
    x[400:601] = 1.0 - np.abs(np.arange(400, 601) - 500) / 100.0
    p, w = find_peaks(x, 0.5, 0.0)
    assert p.tolist() == [500]
    assert abs(w[0] - 100.0) < 1e-12
    assert find_peaks(x, 0.5, 100.5)[0].size == 0   # a width of 100 fails a minimum of 100.5


def test_plateau_middle_and_edges():
    x = np.array([0, 1, 3, 3, 3, 3, 1, 0, 5, 5, 0, 2.0])
    p, _ = find_peaks(x, -1.0, 0.0)
    assert p.tolist() == [3, 8]        # plateau 2..5 -> 3 (rounded down); plateau 8..9 -> 8; the last sample is no peak
    assert find_peaks(np.array([5.0, 1, 5]), 0.0, 0.0)[0].size == 0   # end samples are never peaks
    assert find_peaks(np.array([1.0, 2, 2]), 0.0, 0.0)[0].size == 0   # plateau touching the end


def test_coincidence_brute_force():
    rng = np.random.default_rng(4)
    for _ in range(50):
        lists = [np.sort(rng.choice(20000, int(rng.integers(0, 30)), replace=False)) for _ in range(int(rng.integers(1, 5)))]
        wnd = int(rng.integers(0, 3000))
        ev = coincident_events(lists, wnd)
        want = [int(t) for t in lists[0] if all(any(abs(int(u) - int(t)) <= wnd for u in q) for q in lists[1:])]
        assert ev == want
    assert coincident_events([[100, 5000], [2148], [1, 99]], 2048) == [100]
    assert coincident_events([[100], []], 2048) == []
