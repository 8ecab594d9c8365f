"""Pins of the oracle's intrinsic pre-selection (Sec. IV D; App. B eqs.
dh_itop, x_ML, single_det_ML) against facts fixed by the mathematics: a
noise-free injection, brute-force least squares, the 22-mode closed form,
the edge-on degenerate case and the selection rule.  None of them re-types
the oracle's formulas: the injection comes from the independent forward
simulator, the least squares from numpy's solver on the stacked real system,
the closed form from the complex inner product."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from synth import workload as W


def _setup(seed, modes, dets="HLV", n_bins=64):
    rng = np.random.default_rng(seed)
    net = W.network(dets)
    f = W.freq_bins(n_bins)
    w = W.psd_weights(f, net)
    mc, q, chi = W.draw_intrinsic(rng, 3, (8.0, 30.0), (0.2, 1.0), (-0.5, 0.5))
    h = W.waveform_modes(f, mc, q, chi, modes)
    return rng, net, f, w, h


def _arrival(net, ext1):
    la, lo = ext1["lat"], ext1["lon"]
    n = np.array([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)])
    return ext1["t_geo"] - net.r @ n / 299792458.0


@pytest.mark.parametrize("modes", [W.MODES_HM, W.MODES_22])
def test_noise_free_injection_reaches_rho2_over_2(modes):
    """Data equal to the bank row's own signal in every detector: each
    detector's strain lies in the span of {h_+, h_x} shifted to its arrival
    time, so at the true grid point (phase, time) the single-detector
    maximum is (d_k|d_k)/2, and nowhere on the grid is it larger (a
    projection never exceeds the data's norm)."""
    rng, net, f, w, h = _setup(3, modes)
    n_phi, n_t, dt, j_star, o_star = 8, 7, 2.5e-4, 4, 3
    ext1 = {k: v[0] for k, v in W.draw_extrinsic(rng, 1).items()}
    ext1["cos_iota"] = 0.37
    phi = 2 * np.pi * o_star / n_phi
    d = W.simulate_strain(h[0], modes, f, net, ext1, phi, 400.0)
    tk = _arrival(net, ext1)
    t0 = tk - j_star * dt
    for k in range(len(net.names)):
        times = t0[k] + dt * np.arange(n_t)
        ml = O.single_detector_ml(h[0], modes, ext1["cos_iota"], f, d[k], w[k], times, n_phi)
        half_dd = 0.5 * float(np.sum(w[k] * np.abs(d[k]) ** 2))
        assert ml[o_star, j_star] == pytest.approx(half_dd, rel=1e-10)
        assert np.max(ml) <= half_dd * (1 + 1e-10)
    lnl, per = O.incoherent_ml(h[:1], modes, [ext1["cos_iota"]], f, d, w, t0, dt, n_t, n_phi)
    assert lnl[0] == pytest.approx(0.5 * float(np.sum(w * np.abs(d) ** 2)), rel=1e-10)


def test_brute_force_least_squares():
    """eq. (x_ML): the best real amplitudes minimise the weighted residual
    sum_b w |d - x_+ h_+ - x_x h_x|^2; the likelihood gained is half the
    drop of that residual from (d|d).  Solved here per grid point with
    numpy's least squares on the stacked real and imaginary parts."""
    rng, net, f, w, h = _setup(5, W.MODES_HM, dets="H", n_bins=16)
    d = (rng.standard_normal(16) + 1j * rng.standard_normal(16)) / np.sqrt(w[0])
    ci, n_phi = -0.6, 4
    times = np.array([-1e-3, 0.0, 2e-3])
    ml = O.single_detector_ml(h[1], W.MODES_HM, ci, f, d, w[0], times, n_phi)
    # forward model of each polarisation, written out per channel
    ms = [m for _, m in W.MODES_HM]
    sw = np.sqrt(w[0])
    for o in range(n_phi):
        phi = 2 * np.pi * o / n_phi
        hp = np.zeros(16, complex)
        hx = np.zeros(16, complex)
        for c, (l, m) in enumerate(W.MODES_HM):
            yn, yp = W._swsh_m2(l, -m, ci), W._swsh_m2(l, m, ci)
            hp += 0.5 * (yn + (-1) ** l * yp) * h[1, c] * np.exp(-1j * ms[c] * phi)
            hx += 0.5j * (yn - (-1) ** l * yp) * h[1, c] * np.exp(-1j * ms[c] * phi)
        for j, t in enumerate(times):
            sh = np.exp(-2j * np.pi * f * t)
            A = np.stack([hp * sh * sw, hx * sh * sw], axis=1)
            Ar = np.concatenate([A.real, A.imag])
            y = np.concatenate([(d * sw).real, (d * sw).imag])
            x, *_ = np.linalg.lstsq(Ar, y, rcond=None)
            res = y - Ar @ x
            gain = 0.5 * (y @ y - res @ res)
            assert ml[o, j] == pytest.approx(gain, rel=1e-9, abs=1e-9)


def test_22_mode_closed_form():
    """With the (2,2) mode alone, h_+ and h_x are real and imaginary
    multiples of one complex template, so the fit is a free complex
    amplitude: ln L^ML = |sum_b w d conj(h_22) e^{2 pi i f t}|^2 /
    (2 (h_22|h_22)) at every phase (Cauchy-Schwarz in the complex inner
    product)."""
    rng, net, f, w, h = _setup(7, W.MODES_22, dets="L")
    d = (rng.standard_normal(len(f)) + 1j * rng.standard_normal(len(f))) / np.sqrt(w[0]) + 30 * h[2, 0]
    times = np.array([-2e-3, 0.0, 1e-3, 5e-3])
    ml = O.single_detector_ml(h[2], W.MODES_22, 0.3, f, d, w[0], times, 6)
    hh = float(np.sum(w[0] * np.abs(h[2, 0]) ** 2))
    for j, t in enumerate(times):
        c = np.sum(w[0] * d * np.conj(h[2, 0]) * np.exp(2j * np.pi * f * t))
        assert np.allclose(ml[:, j], abs(c) ** 2 / (2 * hh), rtol=1e-10)


def test_edge_on_22_is_one_polarisation():
    """cos(iota) = 0: the (2,2) mode's cross polarisation vanishes, the fit
    has one real amplitude and ln L^ML = (d|h_+)^2 / (2 (h_+|h_+)) (the
    pseudo-inverse drops the empty direction; no division by zero)."""
    rng, net, f, w, h = _setup(9, W.MODES_22, dets="H")
    d = (rng.standard_normal(len(f)) + 1j * rng.standard_normal(len(f))) / np.sqrt(w[0])
    ml = O.single_detector_ml(h[0], W.MODES_22, 0.0, f, d, w[0], np.array([0.0]), 4)
    kp = 0.5 * (W._swsh_m2(2, -2, 0.0) + W._swsh_m2(2, 2, 0.0))
    for o in range(4):
        hp = kp * h[0, 0] * np.exp(-2j * 2 * np.pi * o / 4)
        b = np.real(np.sum(w[0] * d * np.conj(hp)))
        assert ml[o, 0] == pytest.approx(b * b / (2 * np.sum(w[0] * np.abs(hp) ** 2)), rel=1e-10)
    assert np.all(np.isfinite(ml))


def test_selection_rule():
    """Sec. IV D: keep the rows within delta of the largest incoherent
    maximum, in row order."""
    v = np.array([3.0, 50.0, 29.9, 30.0, 45.0, -1.0])
    assert list(O.preselect(v, 20.0)) == [1, 3, 4]
    assert list(O.preselect(v, 100.0)) == list(range(6))
