"""Pins for the whitening oracle: SciPy's Welch estimator (a library routine the definition reduces
to), closed forms (bin-centred sinusoids, a flat PSD), a brute-force DFT on a tiny stream, and the
statistics of whitened coloured noise."""
import numpy as np
import pytest
import scipy.signal

from oracle.whiten import hann, n_segments, unit_std, welch_psd, welch_psd_stream, whiten, whiten_stream
from paper_2201_11133_amd.synth import coloured_stream

FS = 4096.0


@pytest.mark.parametrize("L,n", [(5000, 256), (4096, 4096), (65536 + 77, 1024), (300, 16)])
def test_welch_is_scipy_welch(L, n):
    x = np.random.default_rng(L).standard_normal(L)
    _, ref = scipy.signal.welch(x, fs=FS, window="hann", nperseg=n, noverlap=n // 2, detrend=False,
                                scaling="density", average="mean", return_onesided=True)
    got = welch_psd(x, FS, n)
    assert got.shape == ref.shape
    assert np.allclose(got, ref, rtol=1e-12, atol=0)


def test_segment_count_and_window():
    assert n_segments(256, 256) == 1
    assert n_segments(256 + 127, 256) == 1
    assert n_segments(256 + 128, 256) == 2
    assert n_segments(255, 256) == 0
    assert np.allclose(hann(8), scipy.signal.get_window("hann", 8), rtol=0, atol=1e-15)
    assert hann(8)[0] == 0.0 and abs(hann(8)[4] - 1.0) < 1e-15          # periodic: peak at n/2


@pytest.mark.parametrize("k0", [2, 37, 126])
def test_welch_sinusoid_total_power(k0):
    """A Hann-windowed sinusoid on bin k0 (2 <= k0 <= n/2 - 2) keeps its mean power A^2/2 in the
    one-sided density summed over bins (Parseval), in every segment."""
    n, L, A = 256, 256 * 9, 1.7
    t = np.arange(L)
    x = A * np.cos(2 * np.pi * k0 * t / n + 0.3)
    P = welch_psd(x, FS, n)
    assert abs(np.sum(P) * FS / n - A * A / 2) < 1e-12
    assert np.argmax(P) == k0


def test_welch_white_noise_level():
    """White noise of variance s^2: the one-sided density is 2 s^2 / fs away from the ends and
    s^2 / fs at zero frequency (no doubling there)."""
    s, n = 1.5, 1024
    x = s * np.random.default_rng(7).standard_normal(1 << 18)
    P = welch_psd(x, FS, n)
    assert abs(np.mean(P[1:-1]) / (2 * s * s / FS) - 1) < 0.02
    assert abs(P[0] / (s * s / FS) - 1) < 0.35


def test_whiten_flat_psd_divides_by_sigma():
    s, n = 2.5, 64
    x = np.random.default_rng(3).standard_normal(1 << 12)
    y = whiten(x, np.full(n // 2 + 1, 2 * s * s / FS), FS, n)
    assert np.allclose(y, x / s, rtol=0, atol=1e-13)


def test_whiten_sinusoid_closed_form():
    """A stream-bin sinusoid comes out scaled by 1 / sqrt(P(f) fs / 2), with P interpolated between
    grid points (bin 100 of 4096 sits at 6.25 on the grid of a 256-point PSD)."""
    L, n, m0, A = 4096, 256, 100, 0.8
    rng = np.random.default_rng(5)
    psd = 1.0 + 0.01 * np.arange(n // 2 + 1) ** 2 + rng.uniform(0, 0.5, n // 2 + 1)
    t = np.arange(L)
    x = A * np.cos(2 * np.pi * m0 * t / L + 1.1)
    p = psd[6] + 0.25 * (psd[7] - psd[6])
    want = A / np.sqrt(p * FS / 2) * np.cos(2 * np.pi * m0 * t / L + 1.1)
    assert np.allclose(whiten(x, psd, FS, n), want, rtol=0, atol=1e-13)


def test_whiten_brute_force_dft():
    """Tiny stream: a full complex DFT written as sums, negative frequencies taking the PSD at |f|."""
    L, n = 64, 16
    rng = np.random.default_rng(11)
    x = rng.standard_normal(L)
    psd = rng.uniform(0.5, 3.0, n // 2 + 1)
    t = np.arange(L)
    Y = np.zeros(L, dtype=complex)
    for m in range(L):
        X = np.sum(x * np.exp(-2j * np.pi * t * m / L))
        pos = min(m, L - m) * n / L                    # grid position of |f|
        j = int(np.floor(pos))
        fr = pos - j
        p = psd[j] if fr == 0 else psd[j] * (1 - fr) + psd[j + 1] * fr
        Y[m] = X / np.sqrt(p * FS / 2)
    y = np.array([np.sum(Y * np.exp(2j * np.pi * tt * np.arange(L) / L)).real / L for tt in t])
    assert np.allclose(whiten(x, psd, FS, n), y, rtol=0, atol=1e-12)


def test_whitened_coloured_noise_is_white():
    """Coloured noise (red component and lines) whitened by its own Welch PSD: the output density
    is flat at 2 / fs (unit variance) at low, middle and line frequencies, where the input's was not."""
    n = 1024
    x = coloured_stream(21, 1 << 18, dtype=np.float64)
    w = whiten_stream(x, FS, n)
    for c in range(2):
        Pin = welch_psd(x[:, c], FS, n)
        Pout = welch_psd(w[:, c], FS, n)
        f = np.arange(n // 2 + 1) * FS / n
        low = (f >= 2) & (f <= 20)
        mid = (f >= 300) & (f <= 1500)
        line = np.argmin(np.abs(f - 60.0))
        assert np.mean(Pin[low]) / np.mean(Pin[mid]) > 5            # the input is coloured
        assert Pin[line] / np.median(Pin[mid]) > 100                 # and has a line
        for band in (low, mid):
            assert abs(np.mean(Pout[band]) * FS / 2 - 1) < 0.1
        assert Pout[line] * FS / 2 < 3
        assert abs(np.std(w[:, c]) - 1) < 1e-12


def test_unit_std_and_scale_invariance():
    x = coloured_stream(22, 1 << 14, dtype=np.float64)
    a = whiten_stream(x, FS, 256)
    b = whiten_stream(x * 1e-21, FS, 256)                           # strain-sized amplitudes
    assert np.allclose(a, b, rtol=1e-9, atol=1e-12)
    assert np.allclose(np.std(a, axis=0), 1.0, rtol=0, atol=1e-13)
    y = np.random.default_rng(1).standard_normal(1000) * 3 + 5
    assert abs(np.std(unit_std(y)) - 1) < 1e-13 and abs(np.mean(unit_std(y)) - np.mean(y) / np.std(y)) < 1e-12   # the mean is kept
    assert welch_psd_stream(x, FS, 256).shape == (2, 129)
