"""Sliding windows over a strain stream, owner-window stitching and the ensemble score (oracle).

Test infrastructure only (see the package docstring).

The paper feeds 1 s windows of two-detector strain at 4096 Hz (Materials and
Methods, "Data preparation") in batches of (1024, 4096, 2) windows and gets one
output per time step of each window ("Optimization with TensorRT"). It does
not say how overlapping windows are combined into one score per sample, nor how
a stream is cut into windows. Readings used here:
  * window k covers samples [k S, k S + W); samples at or past the stream
    length L are zero; n_win = 1 if L <= W else ceil((L - W) / S) + 1;
  * each sample a is scored by its owner window: window 0 for a < W - S,
    otherwise k(a) = floor((a - W + S) / S), at position a - k(a) S (the tail
    S samples of every window after the first);
  * ensemble agreement (Results, "Event Detection": an event is kept only if
    every model reports it) is the per-sample minimum of the members' logits,
    which is >= a threshold exactly when every member's is.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def n_windows(L: int, W: int, S: int) -> int:
    if L <= 0:
        return 0
    if L <= W:
        return 1
    return -(-(L - W) // S) + 1


def gather_windows(u_stream: np.ndarray, W: int, S: int) -> np.ndarray:
    """Materialise all windows of a stream u_stream [L, C] -> [n_win, W, C], zero past L."""
    u_stream = np.asarray(u_stream, dtype=np.float64)
    L, C = u_stream.shape
    n = n_windows(L, W, S)
    out = np.zeros((n, W, C))
    for k in range(n):
        a0 = k * S
        a1 = min(a0 + W, L)
        out[k, :a1 - a0] = u_stream[a0:a1]
    return out


def owner(a: np.ndarray, W: int, S: int) -> Tuple[np.ndarray, np.ndarray]:
    """Owner window index k(a) and in-window position of sample(s) a."""
    a = np.asarray(a, dtype=np.int64)
    k = np.where(a < W - S, 0, (a - W + S) // S)
    return k, a - k * S


def stitch(z_windows: np.ndarray, L: int, W: int, S: int) -> np.ndarray:
    """Per-sample score e[a] = z[k(a)][a - k(a) S] for a in [0, L)."""
    k, pos = owner(np.arange(L), W, S)
    return np.asarray(z_windows, dtype=np.float64)[k, pos]


def ensemble(member_scores: Sequence[np.ndarray]) -> np.ndarray:
    """Per-sample minimum over the members' logits."""
    return np.min(np.stack([np.asarray(s, dtype=np.float64) for s in member_scores]), axis=0)
