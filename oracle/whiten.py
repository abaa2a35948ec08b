"""Whitening front end (oracle): Welch PSD, whitening by the PSD, unit standard deviation.

Test infrastructure only (see the package docstring).

Before the networks see any strain, the paper estimates the power spectral density (PSD) of the
detector data, whitens the strain (and the modeled waveforms) with it, and scales the network input
to unit standard deviation (Materials and Methods, "Data preparation"). It takes the PSD from the
Gravitational Wave Open Science Center's open-source tools, whose standard estimator is Welch's
averaged periodogram. The paper's data segments are 4096 s long at 4096 Hz, i.e. 2^24 samples per
detector ("Advanced LIGO data").

Definitions, for one channel x[t], t in [0, L), sample rate fs:

  Welch PSD over segments of n = nperseg samples with step n/2 (K = floor((L - n) / (n/2)) + 1 full
  segments), periodic Hann window w[j] = 1/2 - 1/2 cos(2 pi j / n), no detrending, mean over the
  segments, one-sided density:
      X_s[k] = sum_j w[j] x[s n/2 + j] exp(-2 pi i j k / n),           k = 0 .. n/2
      P[k]   = c_k / (K fs S2) sum_s |X_s[k]|^2,   S2 = sum_j w[j]^2,  c_k = 1 at k = 0 and n/2, else 2

  Whitening as one transform over the whole stream (L a power of two, n <= L):
      X[m] = sum_t x[t] exp(-2 pi i t m / L),                          m = 0 .. L/2
      P(f_m): P linearly interpolated at f_m = m fs / L between its grid points k fs / n
      Y[m] = X[m] / sqrt(P(f_m) fs / 2)
      y    = the real inverse transform of Y (length L)
  so that white noise of variance s^2, whose one-sided density is 2 s^2 / fs, comes out with unit
  variance.

  Unit standard deviation: out[t] = y[t] / sigma with sigma^2 = (1/L) sum_t (y[t] - mean(y))^2 (the
  mean is not removed).
"""
from __future__ import annotations

from typing import Optional

import numpy as np


def hann(n: int) -> np.ndarray:
    """Periodic Hann window of n points."""
    j = np.arange(n, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * j / n)


def n_segments(L: int, nperseg: int) -> int:
    """Number of full Welch segments of nperseg samples at step nperseg / 2."""
    step = nperseg // 2
    return 0 if L < nperseg else (L - nperseg) // step + 1


def welch_psd(x: np.ndarray, fs: float, nperseg: int) -> np.ndarray:
    """One-sided Welch PSD of one channel: [nperseg / 2 + 1] float64 (the definition above)."""
    x = np.asarray(x, dtype=np.float64)
    K = n_segments(len(x), nperseg)
    if K < 1:
        raise ValueError("stream shorter than one segment")
    w = hann(nperseg)
    step = nperseg // 2
    acc = np.zeros(nperseg // 2 + 1)
    for s in range(K):
        X = np.fft.rfft(w * x[s * step: s * step + nperseg])
        acc += np.abs(X) ** 2
    c = np.full(nperseg // 2 + 1, 2.0)
    c[0] = 1.0
    c[-1] = 1.0
    return c * acc / (K * fs * np.sum(w * w))


def psd_at(psd: np.ndarray, fs: float, nperseg: int, f: np.ndarray) -> np.ndarray:
    """The PSD linearly interpolated at frequencies f (Hz) between its grid points k fs / nperseg."""
    grid = np.arange(nperseg // 2 + 1, dtype=np.float64) * fs / nperseg
    return np.interp(f, grid, psd)


def whiten(x: np.ndarray, psd: np.ndarray, fs: float, nperseg: int) -> np.ndarray:
    """Whitened channel (before the unit-deviation scaling): float64 [L]."""
    x = np.asarray(x, dtype=np.float64)
    L = len(x)
    X = np.fft.rfft(x)
    f = np.arange(L // 2 + 1, dtype=np.float64) * fs / L
    Y = X / np.sqrt(psd_at(psd, fs, nperseg, f) * fs / 2.0)
    return np.fft.irfft(Y, n=L)


def unit_std(y: np.ndarray) -> np.ndarray:
    """y divided by its population standard deviation."""
    y = np.asarray(y, dtype=np.float64)
    return y / np.sqrt(np.mean((y - np.mean(y)) ** 2))


def welch_psd_stream(x2: np.ndarray, fs: float, nperseg: int) -> np.ndarray:
    """PSD of both channels of a [L, 2] stream: [2, nperseg / 2 + 1]."""
    return np.stack([welch_psd(x2[:, c], fs, nperseg) for c in range(2)])


def whiten_stream(x2: np.ndarray, fs: float, nperseg: int, psd: Optional[np.ndarray] = None,
                  normalize: bool = True) -> np.ndarray:
    """Whitened [L, 2] stream (float64); the PSD comes from the stream itself when not given."""
    if psd is None:
        psd = welch_psd_stream(x2, fs, nperseg)
    out = np.empty((x2.shape[0], 2))
    for c in range(2):
        y = whiten(x2[:, c], psd[c], fs, nperseg)
        out[:, c] = unit_std(y) if normalize else y
    return out
