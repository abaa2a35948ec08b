"""Pins for the synthetic input generator: leading-order chirp closed forms, SNR, delays, seeds."""
import math

import numpy as np

from paper_2201_11133_amd import synth


def test_chirp_frequency_is_phase_derivative():
    mc = synth.chirp_mass_for_duration(1.0)
    tau = np.linspace(0.01, 1.0, 2000)
    h = 1e-7
    dphi_dt = -(synth.chirp_phase(tau + h, mc, 0.3) - synth.chirp_phase(tau - h, mc, 0.3)) / (2 * h)
    np.testing.assert_allclose(dphi_dt, 2 * math.pi * synth.chirp_frequency(tau, mc), rtol=1e-6)


def test_duration_and_band_edges():
    for tau20 in [0.2, 0.7, 2.0]:
        mc = synth.chirp_mass_for_duration(tau20)
        assert abs(synth.tau_at_frequency(20.0, mc) - tau20) < 1e-12 * max(1, tau20)
        assert abs(synth.chirp_frequency(np.array([tau20]), mc)[0] - 20.0) < 1e-9
        t300 = synth.tau_at_frequency(300.0, mc)
        assert abs(synth.chirp_frequency(np.array([t300]), mc)[0] - 300.0) < 1e-7
        assert t300 < 2e-3
    # chirp mass in solar masses spans about 16.8 - 66.7
    msun_s = 4.925490947e-6
    assert 16 < synth.chirp_mass_for_duration(2.0) / msun_s < 17.5
    assert 65 < synth.chirp_mass_for_duration(0.2) / msun_s < 68


def test_snr_normalisation_and_delay():
    rng = np.random.default_rng(0)
    inj = synth.draw_injection(rng, 1.5)
    sig = synth.injection_signal(inj, 0.0, 3 * synth.FS)
    assert abs(math.sqrt(float(np.sum(sig * sig))) - inj.rho) < 1e-9
    # Livingston channel is Hanford's waveform delayed by delta, evaluated analytically
    t = np.arange(3 * synth.FS) / synth.FS
    h0 = synth.chirp_waveform(t, inj.tc, inj.mc, inj.phi_c)
    h1 = synth.chirp_waveform(t - inj.delta, inj.tc, inj.mc, inj.phi_c)
    scale = sig[:, 0][np.argmax(np.abs(h0))] / h0[np.argmax(np.abs(h0))]
    np.testing.assert_allclose(sig[:, 0], h0 * scale, atol=1e-12)
    np.testing.assert_allclose(sig[:, 1], h1 * scale, atol=1e-12)


def test_signal_confined_to_band_window():
    rng = np.random.default_rng(1)
    inj = synth.draw_injection(rng, 2.5)
    t = np.arange(4 * synth.FS) / synth.FS
    h = synth.chirp_waveform(t, inj.tc, inj.mc, inj.phi_c)
    nz = np.nonzero(h)[0]
    assert t[nz[0]] >= inj.tc - inj.tau20 - 1e-12
    assert t[nz[-1]] <= inj.tc


def test_streams_reproducible_and_spaced():
    x1, i1 = synth.make_stream(101, 120.0, 8)
    x2, i2 = synth.make_stream(101, 120.0, 8)
    assert np.array_equal(x1, x2) and [j.tc for j in i1] == [j.tc for j in i2]
    tcs = sorted(j.tc for j in i1)
    assert len(tcs) == 8 and np.all(np.diff(tcs) >= 10.0 - 1e-9)
    assert tcs[0] >= 4.0 and tcs[-1] <= 116.0
    assert x1.shape == (120 * 4096, 2) and x1.dtype == np.float32
    # noise is close to unit variance
    assert abs(float(np.std(x1)) - 1.0) < 0.01


def test_windows_and_labels():
    x, injs = synth.make_windows(100, 64, 8)
    assert x.shape == (64, 4096, 2) and len(injs) == 8
    for i, inj in injs:
        assert 0.25 <= inj.tc <= 0.9
    y = synth.box_labels(4096, 0.5)
    assert y.sum() == np.count_nonzero(np.abs(np.arange(4096) / 4096 - 0.5) <= 0.1)
    assert synth.box_labels(10, None).sum() == 0


def test_ragged_lengths_range():
    L = synth.ragged_lengths(103, 32)
    assert len(L) == 32 and min(L) >= 8 * 4096 and max(L) <= 4096 * 4096
