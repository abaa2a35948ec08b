"""Time-slide background and false-alarm rate (oracle).

Test infrastructure only (see the package docstring).

The paper estimates how often the ensemble fires on noise by building one to
five years of background from its month of two-detector data with time slides
(Results, "Statistical Analysis"): one detector's strain is shifted in time
against the other's by far more than the inter-detector light travel time, so
no astrophysical coincidence survives, and every trigger found in the slid data
counts as a false positive. The paper reports the counts per slid dataset
(about 1.3 per month); the false-alarm rate is such a count divided by the slid
live time.

Readings taken here (the paper points to its reference for the shifting
procedure and does not restate it):
  - the shift is circular over the stream, channel 1 moves and channel 0 stays:
        slid[t, 0] = x[t, 0],   slid[t, 1] = x[(t + s) mod L, 1];
  - the false-alarm curve over thresholds comes from one trigger list found at
    the lowest threshold: the clustering condition does not involve the
    threshold, so raising it only removes records whose score falls below it.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def time_slide(x: np.ndarray, shift: int) -> np.ndarray:
    """Slid copy of a [L, 2] two-channel stream: channel 1 read `shift` samples later, circularly."""
    x = np.asarray(x)
    L = x.shape[0]
    out = x.copy()
    if L == 0:
        return out
    s = int(shift) % L
    out[:, 1] = np.concatenate([x[s:, 1], x[:s, 1]])
    return out


def far_curve(trigger_logits: Sequence[float], thresholds: Sequence[float],
              livetime_s: float) -> Tuple[np.ndarray, np.ndarray]:
    """(counts, rate per second): records with logit >= each threshold, over the slid live time."""
    z = np.asarray(trigger_logits, dtype=np.float64)
    counts = np.array([int(np.sum(z >= float(t))) for t in thresholds], dtype=np.int64)
    return counts, counts / float(livetime_s)
