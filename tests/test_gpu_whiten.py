"""Whitening front end on the GPU against the oracle: the Welch PSD and the whitened, unit-deviation
stream, element by element, at sizes from the minimum to a 4096 s stream, with bounds derived from
the float32 transforms.

Bounds (u = 2^-24 the float32 unit roundoff, eta = 6u the per-stage error of a radix-2 butterfly
with rounded twiddles, the standard FFT forward-error analysis, Higham, "Accuracy and Stability of
Numerical Algorithms", ch. 24):
  - a transform of length n moves ||dZ||_2 <= (log2 n + 2) eta ||Z||_2 (two more stages' worth for
    the four-step twiddle and the windowing);
  - Welch, per segment and bin: |dX_k| <= E_s = (log2 n + 2) eta sqrt(n) ||z_s||_2, so
    |dP_k| <= c_k scale sum_s (2 |X_s,k| E_s + E_s^2) and, by Cauchy-Schwarz,
    sum_s |X_s,k| <= K sqrt(mean_s |X_s,k|^2);
  - whitening: the forward error is multiplied by at most the largest coefficient, the inverse adds
    its own, and the coefficient product 4u; the L2 norm over time bounds every element.
"""
import math

import numpy as np
import pytest

from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FS = 4096.0
U = 2.0 ** -24
ETA = 6 * U


@pytest.fixture(scope="module")
def g():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_11133_amd import gwd
    return gwd


def welch_bound(x, n, psd64):
    """Per (channel, bin) bound on |P_gpu - P_oracle| (see the module docstring)."""
    from oracle.whiten import hann, n_segments
    L = x.shape[0]
    K = n_segments(L, n)
    w = hann(n)
    step = n // 2
    zmax = 0.0
    for s in range(K):
        seg = x[s * step: s * step + n].astype(np.float64) * w[:, None]
        zmax = max(zmax, math.sqrt(float(np.sum(seg * seg))))
    E = (math.log2(n) + 2) * ETA * math.sqrt(n) * zmax
    scale = 1.0 / (K * FS * np.sum(w * w))
    c = np.full(n // 2 + 1, 2.0)
    c[0] = c[-1] = 1.0
    mean_sq = psd64 / (c * scale)                     # mean_s |X_s,k|^2
    return c * scale * K * (2 * np.sqrt(mean_sq) * E + E * E) + 1e-12 * psd64


def whiten_bound(x, psd64, n, y64):
    """L2 (over time and channels) bound on the error of the unnormalised whitened stream."""
    from oracle.whiten import psd_at
    L = x.shape[0]
    lg = math.log2(L)
    f = np.arange(L // 2 + 1) * FS / L
    amax = max(float(np.max(1 / np.sqrt(psd_at(psd64[c], FS, n, f) * FS / 2))) for c in range(2))
    zn = math.sqrt(float(np.sum(x.astype(np.float64) ** 2)))
    yn = math.sqrt(float(np.sum(y64 ** 2)))
    return amax * (lg + 2) * ETA * zn + ((lg + 2) * ETA + 4 * U) * yn


def run_case(g, x, n, planar=False):
    from oracle.whiten import welch_psd_stream, whiten_stream
    xd = to_dev(x)
    src = (to_dev(x[:, 0].copy()), to_dev(x[:, 1].copy())) if planar else xd
    psd = g.welch_psd(src, n, FS)
    out = g.whiten(src, psd, n, FS, True)
    raw = g.whiten(src, psd, n, FS, False)
    torch.cuda.synchronize()
    psd_g = psd.cpu().numpy()
    psd_o = welch_psd_stream(x.astype(np.float64), FS, n)
    dp = np.abs(psd_g - psd_o)
    bp = np.stack([welch_bound(x, n, psd_o[c]) for c in range(2)])   # both channels share a transform
    assert np.all(dp <= bp), float(np.max(dp / bp))
    # whitening by the oracle's PSD would hide nothing: both sides whiten by the GPU's own PSD
    y_o = whiten_stream(x.astype(np.float64), FS, n, psd=psd_g, normalize=False)
    w_o = whiten_stream(x.astype(np.float64), FS, n, psd=psd_g, normalize=True)
    b = whiten_bound(x, psd_g, n, y_o)
    d_raw = raw.cpu().numpy().astype(np.float64) - y_o
    assert math.sqrt(float(np.sum(d_raw ** 2))) <= b
    sig = np.std(y_o, axis=0)
    bn = b / float(np.min(sig)) + 4 * U * math.sqrt(float(np.sum(w_o ** 2)))
    d = out.cpu().numpy().astype(np.float64) - w_o
    assert math.sqrt(float(np.sum(d ** 2))) <= bn
    print(f"  L={x.shape[0]} n={n}: psd max rel {float(np.max(dp / psd_o)):.2e}, "
          f"whitened max |d| {float(np.max(np.abs(d))):.2e} (L2 bound {bn:.2e})", flush=True)
    return out


@pytest.mark.parametrize("logl,n", [(4, 16), (13, 256), (16, 1024), (16, 65536 // 16), (20, 16384)])
def test_whiten_matches_oracle(g, logl, n):
    from paper_2201_11133_amd.synth import coloured_stream
    print(f"case: whiten L=2^{logl} n={n}", flush=True)
    x = coloured_stream(300 + logl, 1 << logl)
    run_case(g, x, n)


def test_whiten_planar_strain_scale(g):
    """Two separate channel buffers and strain-sized amplitudes (1e-21): same whitened stream as the
    unit-scale interleaved input, up to the bound."""
    from paper_2201_11133_amd.synth import coloured_stream
    print("case: whiten planar 1e-21", flush=True)
    x = coloured_stream(77, 1 << 15, scale=1e-21)
    out = run_case(g, x, 512, planar=True)
    ref = run_case(g, coloured_stream(77, 1 << 15), 512)
    assert float(torch.max(torch.abs(out - ref))) < 1e-3


def test_whiten_in_place_and_ragged_welch(g):
    from oracle.whiten import welch_psd_stream
    from paper_2201_11133_amd.synth import coloured_stream
    print("case: whiten in place, Welch on a ragged length", flush=True)
    x = coloured_stream(5, 1 << 14)
    xd = to_dev(x)
    psd = g.welch_psd(xd, 256, FS)
    want = g.whiten(xd, psd, 256, FS, True).clone()
    g.whiten(xd, psd, 256, FS, True, out=xd)            # the source's own buffer
    assert torch.equal(xd, want)
    xr = coloured_stream(6, 100003)
    pr = g.welch_psd(to_dev(xr), 1024, FS).cpu().numpy()
    po = welch_psd_stream(xr.astype(np.float64), FS, 1024)
    bp = np.stack([welch_bound(xr, 1024, po[c]) for c in range(2)])
    assert np.all(np.abs(pr - po) <= bp)


def test_whiten_full_segment(g):
    """A 4096 s two-detector segment (2^24 samples per channel, the paper's segment length) with
    4 s Welch segments: the workload the benchmark times."""
    from paper_2201_11133_amd.synth import coloured_stream
    print("case: whiten 4096 s", flush=True)
    x = coloured_stream(2024, 1 << 24)
    run_case(g, x, 16384)


def test_whiten_large_transform(g):
    """2^25 samples: columns of 8192 points (the 128 KB LDS variant of the column passes)."""
    from paper_2201_11133_amd.synth import coloured_stream
    print("case: whiten 2^25", flush=True)
    x = coloured_stream(2025, 1 << 25)
    run_case(g, x, 4096)
