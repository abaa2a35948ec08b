"""Seeded synthetic inputs: white-noise strain with leading-order chirps, He-normal weights, labels.

This module only draws inputs. It holds none of the classifier's arithmetic and
is the one module that both the HIP path's callers and the oracle's tests use.

Stand-ins for the paper's data (Materials and Methods, "Modeled waveforms",
"Advanced LIGO data", "Data preparation"): the paper whitens real detector
strain and injects SEOBNRv3 waveforms at a range of signal-to-noise ratios,
normalising the result to unit standard deviation, at 4096 Hz. Here the
whitened noise is i.i.d. N(0, 1) and the waveform is the leading-order
(Newtonian, quadrupole) inspiral chirp:

  tau = t_c - t (seconds), Mc = chirp mass in seconds (G Mc / c^3)
  f(tau)   = (1 / 8 pi) (5 / tau)^(3/8) Mc^(-5/8)
  phi(tau) = phi_c - 2 (tau / (5 Mc))^(5/8)          so d phi / dt = 2 pi f
  h(t)     = A tau^(-1/4) cos phi(tau)

kept between f = 20 Hz and f = 300 Hz, with a 0.05 s half-Hann taper at the
start. The in-band duration tau20 ~ U[0.2, 2] s fixes Mc. The Livingston
channel is the same waveform delayed by delta ~ U[-10, 10] ms (evaluated
analytically). A is set so that the network optimal SNR
sqrt(sum over both channels and all samples of h^2) equals rho ~ U[8, 20].
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

FS = 4096                       # samples per second
F_LO, F_HI = 20.0, 300.0
TAPER_S = 0.05


# ---------------------------------------------------------------- chirp
def chirp_mass_for_duration(tau20: float) -> float:
    """Chirp mass (seconds) whose 20 Hz -> coalescence time is tau20."""
    return (tau20 / ((5.0 / 256.0) * (20.0 * math.pi) ** (-8.0 / 3.0))) ** (-3.0 / 5.0)


def tau_at_frequency(f: float, mc: float) -> float:
    """Time before coalescence at which the leading-order frequency equals f."""
    return 5.0 * (8.0 * math.pi * f) ** (-8.0 / 3.0) * mc ** (-5.0 / 3.0)


def chirp_frequency(tau: np.ndarray, mc: float) -> np.ndarray:
    return (1.0 / (8.0 * math.pi)) * (5.0 / tau) ** (3.0 / 8.0) * mc ** (-5.0 / 8.0)


def chirp_phase(tau: np.ndarray, mc: float, phi_c: float) -> np.ndarray:
    return phi_c - 2.0 * (tau / (5.0 * mc)) ** (5.0 / 8.0)


def chirp_waveform(t: np.ndarray, tc: float, mc: float, phi_c: float) -> np.ndarray:
    """Unit-amplitude band-limited chirp evaluated at times t (seconds)."""
    t = np.asarray(t, dtype=np.float64)
    tau = tc - t
    t20 = tau_at_frequency(F_LO, mc)
    t300 = tau_at_frequency(F_HI, mc)
    inband = (tau <= t20) & (tau >= t300)
    out = np.zeros_like(t)
    ti = tau[inband]
    w = ti ** (-0.25) * np.cos(chirp_phase(ti, mc, phi_c))
    # half-Hann rising taper over the first TAPER_S seconds of the band
    since_start = t20 - ti
    taper = np.where(since_start < TAPER_S, 0.5 * (1.0 - np.cos(math.pi * since_start / TAPER_S)), 1.0)
    out[inband] = w * taper
    return out


@dataclass
class Injection:
    tc: float          # coalescence time in the stream (s, Hanford)
    tau20: float       # in-band duration (s)
    mc: float          # chirp mass (s)
    phi_c: float
    delta: float       # Livingston delay (s)
    rho: float         # network optimal SNR


def draw_injection(rng: np.random.Generator, tc: float) -> Injection:
    tau20 = rng.uniform(0.2, 2.0)
    return Injection(tc=tc, tau20=tau20, mc=chirp_mass_for_duration(tau20),
                     phi_c=rng.uniform(0.0, 2.0 * math.pi), delta=rng.uniform(-0.010, 0.010),
                     rho=rng.uniform(8.0, 20.0))


def injection_signal(inj: Injection, t0: float, n: int) -> np.ndarray:
    """Two-channel signal [n, 2] on samples t0 + i / FS, scaled to the network SNR rho."""
    t = t0 + np.arange(n) / FS
    h = np.stack([chirp_waveform(t, inj.tc, inj.mc, inj.phi_c),
                  chirp_waveform(t - inj.delta, inj.tc, inj.mc, inj.phi_c)], axis=1)
    norm = math.sqrt(float(np.sum(h * h)))
    return h * (inj.rho / norm) if norm > 0 else h


def _support(inj: Injection) -> Tuple[float, float]:
    """Time interval (s) that contains the injection's nonzero samples in both channels."""
    return inj.tc - inj.tau20 - 0.02, inj.tc + 0.02


def add_injection(stream: np.ndarray, inj: Injection, t_offset: float = 0.0) -> None:
    """Add inj to stream [L, 2] (in place); stream sample i is at time t_offset + i / FS."""
    lo, hi = _support(inj)
    i0 = max(0, int(math.floor((lo - t_offset) * FS)))
    i1 = min(stream.shape[0], int(math.ceil((hi - t_offset) * FS)) + 1)
    if i1 <= i0:
        return
    full = injection_signal(inj, t_offset + i0 / FS, i1 - i0)
    stream[i0:i1] += full.astype(stream.dtype)


def place_times(rng: np.random.Generator, n: int, t_total: float, margin: float, spacing: float) -> List[float]:
    """n uniform times in [margin, t_total - margin] with pairwise spacing >= spacing (fewer if they do not fit)."""
    span = t_total - 2 * margin
    while n > 0 and span - (n - 1) * spacing < 0:
        n -= 1
    if n == 0:
        return []
    free = span - (n - 1) * spacing
    base = np.sort(rng.uniform(0.0, free, size=n))
    return [float(margin + b + i * spacing) for i, b in enumerate(base)]


# ---------------------------------------------------------------- streams and windows
def noise_stream(rng: np.random.Generator, L: int, dtype=np.float32) -> np.ndarray:
    return rng.standard_normal((L, 2), dtype=np.float32 if dtype == np.float32 else np.float64).astype(dtype, copy=False)


def coloured_stream(seed: int, L: int, scale: float = 1.0, dtype=np.float32) -> np.ndarray:
    """Two-channel coloured noise [L, 2], a stand-in for unwhitened detector strain: per channel a
    red component (white noise through a one-pole low-pass, pole 0.99, gain 0.1), a white floor of
    unit variance, and power-line-like sinusoids (channel 0: 60 Hz amplitude 3 and 120 Hz amplitude
    1; channel 1: 60 Hz amplitude 2 and 180 Hz amplitude 1) with random phases, all times `scale`."""
    from scipy.signal import lfilter
    rng = np.random.default_rng(seed)
    t = np.arange(L, dtype=np.float64) / FS
    lines = (((60.0, 3.0), (120.0, 1.0)), ((60.0, 2.0), (180.0, 1.0)))
    x = np.empty((L, 2), dtype=np.float64)
    for c in range(2):
        red = lfilter([0.1], [1.0, -0.99], rng.standard_normal(L))
        x[:, c] = red + rng.standard_normal(L)
        for f, a in lines[c]:
            x[:, c] += a * np.cos(2.0 * np.pi * f * t + rng.uniform(0.0, 2.0 * np.pi))
    return (x * scale).astype(dtype)


def make_stream(seed: int, seconds: float, n_chirps: int, spacing: float = 10.0, margin: float = 4.0,
                dtype=np.float32) -> Tuple[np.ndarray, List[Injection]]:
    """One two-channel stream [L, 2] of white noise with n_chirps leading-order chirps."""
    rng = np.random.default_rng(seed)
    L = int(round(seconds * FS))
    x = noise_stream(rng, L, dtype)
    injs = [draw_injection(rng, tc) for tc in place_times(rng, n_chirps, seconds, margin, spacing)]
    for inj in injs:
        add_injection(x, inj)
    return x, injs


def make_windows(seed: int, n_windows: int, n_chirped: int, W: int = 4096, dtype=np.float32
                 ) -> Tuple[np.ndarray, List[Tuple[int, Injection]]]:
    """n_windows independent windows [n, W, 2]; n_chirped of them (indices drawn from the seed)
    carry a chirp with tc_local ~ U[0.25, 0.9] s."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n_windows, W, 2), dtype=np.float32).astype(dtype, copy=False)
    idx = np.sort(rng.choice(n_windows, size=n_chirped, replace=False)) if n_chirped else np.zeros(0, int)
    injs = []
    for i in idx:
        inj = draw_injection(rng, rng.uniform(0.25, 0.9))
        add_injection(x[i], inj)
        injs.append((int(i), inj))
    return x, injs


def ragged_lengths(seed: int, n_streams: int, lo_s: float = 8.0, hi_s: float = 4096.0) -> List[int]:
    """Stream lengths (samples) log-uniform in [lo_s, hi_s] seconds."""
    rng = np.random.default_rng(seed)
    return [int(round(FS * math.exp(rng.uniform(math.log(lo_s), math.log(hi_s))))) for _ in range(n_streams)]


def box_labels(n: int, tc_local: Optional[float], half_width_s: float = 0.1) -> np.ndarray:
    """Per-timestep training labels: 1 where |t - tc| <= half_width_s, else 0."""
    y = np.zeros(n)
    if tc_local is not None:
        t = np.arange(n) / FS
        y[np.abs(t - tc_local) <= half_width_s] = 1.0
    return y


# ---------------------------------------------------------------- weights
def weight_layout(kind: int, channels: int, skip_channels: int = 128, head_channels: int = 128,
                  n_layers: int = 30, in_channels: int = 2, kernel: int = 2, input_kernel: int = 1
                  ) -> List[Tuple[Tuple[int, ...], int]]:
    """(shape, fan_in) of every tensor of the flat weight blob, in blob order (fan_in 0 = bias).

    This is the generator's own statement of the public blob format.
    """
    out: List[Tuple[Tuple[int, ...], int]] = []
    if kind == 0:
        cin = in_channels
        for _ in range(n_layers):
            out += [((channels, cin, kernel), cin * kernel), ((channels,), 0)]
            cin = channels
        return out + [((1, channels), channels), ((1,), 0)]
    if kind == 2:       # one single-channel gated branch per detector, then the head on both skip sums
        branch = weight_layout(1, channels, skip_channels, head_channels, n_layers, 1, kernel, input_kernel)[:-4]
        return branch + branch + [((head_channels, 2 * skip_channels), 2 * skip_channels), ((head_channels,), 0),
                                  ((1, head_channels), head_channels), ((1,), 0)]
    C, S, H = channels, skip_channels, head_channels
    if input_kernel == 1:
        out.append(((C, in_channels), in_channels))
    else:
        out.append(((C, in_channels, input_kernel), in_channels * input_kernel))
    out.append(((C,), 0))
    for l in range(n_layers):
        out += [((2 * C, C, kernel), C * kernel), ((2 * C,), 0)]
        if l < n_layers - 1:
            out += [((C, C), C), ((C,), 0)]
        out += [((S, C), C), ((S,), 0)]
    out += [((H, S), S), ((H,), 0), ((1, H), H), ((1,), 0)]
    return out


def he_normal_blob(seed: int, layout: Sequence[Tuple[Tuple[int, ...], int]]) -> np.ndarray:
    """Flat float32 blob: weights ~ N(0, 2 / fan_in) (not truncated), biases 0.

    Normals are drawn from default_rng(seed).standard_normal tensor by tensor in
    blob order; biases draw nothing.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for shape, fan_in in layout:
        n = int(np.prod(shape))
        if fan_in == 0:
            parts.append(np.zeros(n))
        else:
            parts.append(rng.standard_normal(n) * math.sqrt(2.0 / fan_in))
    return np.concatenate(parts).astype(np.float32)


TINY_LAYOUT = dict(kind=0, channels=16, n_layers=4)
FULL_LAYOUT = dict(kind=1, channels=128, skip_channels=128, head_channels=128, n_layers=30)
TWO_BRANCH_LAYOUT = dict(kind=2, channels=64, skip_channels=64, head_channels=128, n_layers=30)


def tiny_weights(seed: int = 0) -> np.ndarray:
    return he_normal_blob(seed, weight_layout(**TINY_LAYOUT))


def full_weights(seed: int = 1, **kw) -> np.ndarray:
    lay = dict(FULL_LAYOUT)
    lay.update(kw)
    return he_normal_blob(seed, weight_layout(**lay))


def two_branch_weights(seed: int = 21) -> np.ndarray:
    """He-normal blob of the two-branch member (two 64-channel branches, 128-channel head)."""
    return he_normal_blob(seed, weight_layout(**TWO_BRANCH_LAYOUT))

