"""The paper's post-processing of model outputs (oracle): peak finding and all-member coincidence.

Test infrastructure only (see the package docstring).

The paper runs SciPy's find_peaks on each model's output to locate mergers (Methods, "AI ensemble
construction"). For the ROC study it keeps peaks whose width is at least 0.5 s while the height
threshold is swept from 0 to 0.9998 (Results, "Statistical Analysis"). It flags an event only when
all models report a trigger within 0.5 s of each other (Results, "Event Detection").

find_peaks here IS the library routine (scipy.signal.find_peaks with `height` and `width`, the
default relative height 0.5), so its definition is SciPy's:
  - a peak is a sample, or the middle (rounded down) of a run of equal samples, with a strictly
    lower neighbour on each side; the first and last samples are never peaks;
  - its prominence is its height above the higher of the two lowest points reached when walking
    left and right until a strictly higher sample (or the end);
  - its width is measured at half that prominence below the peak, between the points where the
    signal crosses that level, with linear interpolation between samples, inside the two bases.

Readings taken here (the paper does not spell them out):
  - the peak search runs on each member's probability p = 1 / (1 + e^-z), in float64;
  - coincidence anchors on member 0: a peak of member 0 at sample t is an event when every other
    member has a peak at some t' with |t' - t| <= window (2048 samples = 0.5 s at 4096 Hz); the
    event is reported at t.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np
from scipy.signal import find_peaks as _scipy_find_peaks


def find_peaks(x: np.ndarray, height: float, min_width: float) -> Tuple[np.ndarray, np.ndarray]:
    """(peak sample indices, widths in samples) of x: peaks of height >= height, width >= min_width."""
    x = np.asarray(x, dtype=np.float64)
    peaks, props = _scipy_find_peaks(x, height=height, width=min_width)
    return peaks.astype(np.int64), np.asarray(props["widths"], dtype=np.float64)


def coincident_events(peak_lists: Sequence[Sequence[int]], window: int) -> List[int]:
    """Peaks of member 0 that every other member matches within +/- window samples."""
    if not peak_lists:
        return []
    others = [np.sort(np.asarray(p, dtype=np.int64)) for p in peak_lists[1:]]
    events = []
    for t in peak_lists[0]:
        ok = True
        for q in others:
            if q.size == 0 or np.min(np.abs(q - int(t))) > window:
                ok = False
                break
        if ok:
            events.append(int(t))
    return events
