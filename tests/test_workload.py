"""Checks of the synthetic input recipe (not of the method)."""
import numpy as np
import pytest

from synth import workload as W


def test_noise_whitening():
    """n = (x + i y)/sqrt(w): E sum w|n|^2 = 2 N_b N_k and Re(n|h) ~ N(0, (h|h))."""
    rng = np.random.default_rng(0)
    net = W.network("HLV")
    f = W.freq_bins(256)
    w = W.psd_weights(f, net)
    h = W.waveform_modes(f, np.array([20.0]), np.array([0.7]), np.array([0.1]), W.MODES_22)[0, 0]
    hk = np.stack([h, 0.5 * h, 0.3 * h])
    hh = float(np.sum(w * np.abs(hk) ** 2))
    nn, proj = [], []
    for _ in range(400):
        n = W.noise(rng, w)
        nn.append(np.sum(w * np.abs(n) ** 2))
        proj.append(np.real(np.sum(w * n * np.conj(hk))))
    assert np.mean(nn) == pytest.approx(2 * 256 * 3, rel=0.02)
    assert np.var(proj) / hh == pytest.approx(1.0, rel=0.2)


def test_bins_and_widths():
    f = W.freq_bins(64)
    assert f[0] == pytest.approx(20.0) and f[-1] == pytest.approx(512.0)
    df = W.bin_widths(f)
    assert np.sum(df) == pytest.approx(f[-1] - f[0])


def test_waveform_shapes_and_cutoff():
    f = W.freq_bins(256)
    mc, q, chi = W.draw_intrinsic(np.random.default_rng(1), 50, (5, 80), (0.1, 1), (-0.9, 0.9))
    h = W.waveform_modes(f, mc, q, chi, W.MODES_HM)
    assert h.shape == (50, 5, 256) and h.dtype == np.complex128
    assert np.all(np.isfinite(h))
    # equal-mass sources have no odd-m content
    h1 = W.waveform_modes(f, np.array([10.0]), np.array([1.0]), np.array([0.0]), W.MODES_HM)
    assert np.all(h1[0, 1] == 0) and np.all(h1[0, 2] == 0)


def test_injection_snr():
    wl = W.config_tiny(seed=2, noise_on=False, snr=15.0)
    assert np.sqrt(np.sum(wl.w * np.abs(wl.d) ** 2)) == pytest.approx(15.0, rel=1e-12)
