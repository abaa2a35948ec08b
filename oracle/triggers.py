"""Ensemble-agreement threshold and trigger clustering (oracle).

Test infrastructure only (see the package docstring).

The paper keeps a candidate only when every member of the ensemble reports it
(Results, "Event Detection") and locates mergers by peak finding on the model
outputs ("AI ensemble construction"). The rule used here, with a fixed
threshold probability and clustering window Wc (0.9 and 4096 samples):

  sample a of a stream is a trigger iff
      e[a] >= logit(p_thr)                 (inclusive, compared in logit space), and
      e[a] >  e[b] for every b in [a - Wc, a)  within the stream, and
      e[a] >= e[b] for every b in (a, a + Wc]  within the stream,
  i.e. a +/- Wc non-maximum suppression whose ties go to the earliest sample.

Consequences used as pins: triggers of one stream are at least Wc + 1 samples
apart; a constant stream above threshold triggers exactly at its first sample;
a strictly increasing one at its last sample.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np
from scipy.ndimage import maximum_filter1d

from .forward import sigmoid


def logit_threshold(p_thr: float) -> float:
    """logit(p) = ln(p / (1 - p)); for p = 0.9 this is ln 9."""
    return math.log(p_thr / (1.0 - p_thr))


def _one_stream(e: np.ndarray, thr: float, wc: int) -> np.ndarray:
    """Trigger sample indices of one stream (vectorised; sliding maxima are a library routine)."""
    e = np.asarray(e, dtype=np.float64)
    n = e.size
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    ninf = -np.inf
    # left[a] = max e[b], b in [a - wc, a);  right[a] = max e[b], b in (a, a + wc]
    pad = np.concatenate([np.full(wc, ninf), e, np.full(wc, ninf)])
    win_max = forward_max(pad, wc)          # win_max[i] = max pad[i .. i + wc - 1]
    left = win_max[0:n]                     # pad[a .. a + wc - 1]          = e[a - wc .. a - 1]
    right = win_max[wc + 1:wc + 1 + n]      # pad[a + wc + 1 .. a + 2 wc]   = e[a + 1 .. a + wc]
    ok = (e >= thr) & (e > left) & (e >= right)
    return np.nonzero(ok)[0].astype(np.int64)


def forward_max(pad: np.ndarray, wc: int) -> np.ndarray:
    """max of pad[i .. i + wc - 1] for every i (positions past the end count as -inf)."""
    return maximum_filter1d(pad, size=wc, origin=-(wc // 2), mode="constant", cval=-np.inf)


def triggers(e: np.ndarray, offsets: Sequence[int], p_thr: float = 0.9, wc: int = 4096
             ) -> List[Tuple[int, int, float, float]]:
    """All triggers of streams packed back to back in e, stream s = e[offsets[s]:offsets[s+1]].

    Returns (stream, sample, logit, probability) records sorted by (stream, sample).
    """
    thr = logit_threshold(p_thr)
    out: List[Tuple[int, int, float, float]] = []
    for s in range(len(offsets) - 1):
        seg = np.asarray(e[offsets[s]:offsets[s + 1]], dtype=np.float64)
        for a in _one_stream(seg, thr, wc):
            out.append((s, int(a), float(seg[a]), float(sigmoid(seg[a]))))
    return out


def triggers_brute(e: np.ndarray, offsets: Sequence[int], p_thr: float = 0.9, wc: int = 4096
                   ) -> List[Tuple[int, int]]:
    """Pure-Python O(N Wc) statement of the same rule, for tiny inputs."""
    thr = logit_threshold(p_thr)
    out: List[Tuple[int, int]] = []
    for s in range(len(offsets) - 1):
        seg = [float(v) for v in e[offsets[s]:offsets[s + 1]]]
        n = len(seg)
        for a in range(n):
            if not seg[a] >= thr:
                continue
            if all(seg[a] > seg[b] for b in range(max(0, a - wc), a)) and \
               all(seg[a] >= seg[b] for b in range(a + 1, min(n, a + wc + 1))):
                out.append((s, a))
    return out


def fragile_decisions(e: np.ndarray, offsets: Sequence[int], p_thr: float = 0.9, wc: int = 4096,
                      margin: float = 1e-4) -> set:
    """(stream, sample) pairs whose trigger decision lies within `margin` (in logit) of flipping:
    the score is within margin of the threshold, or of the largest score among its in-stream
    neighbours in [a - wc, a) and (a, a + wc].

    If another computation of the scores differs from e by less than margin / 2 everywhere, its
    trigger list can differ from the one of e only at these samples: each of the three comparisons
    of the rule moves by less than margin.
    """
    thr = logit_threshold(p_thr)
    out = set()
    for s in range(len(offsets) - 1):
        seg = np.asarray(e[offsets[s]:offsets[s + 1]], dtype=np.float64)
        n = seg.size
        if n == 0:
            continue
        pad = np.concatenate([np.full(wc, -np.inf), seg, np.full(wc, -np.inf)])
        win_max = forward_max(pad, wc)
        comp = np.maximum(win_max[0:n], win_max[wc + 1:wc + 1 + n])
        close = (np.abs(seg - thr) < margin) | (np.abs(seg - comp) < margin)
        out.update((s, int(a)) for a in np.nonzero(close)[0])
    return out
