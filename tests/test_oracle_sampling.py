"""Pins of the oracle's posterior sampling (Sec. III B resampling; Sec. V B):
the SplitMix64 generator against its published first output, systematic
resampling's counts, the phase draw on equal weights, and the distance
draw against the closed form of an empty template and against an
independent fine-grid distribution function."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def test_splitmix64_first_output():
    # the first output of SplitMix64 seeded with 0 is 0xe220a8397b1dcdaf
    assert O.splitmix64_uniform(0, 0) == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53
    u = np.array([O.splitmix64_uniform(7, n) for n in range(20000)])
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01


def test_systematic_counts():
    """Each weight is drawn floor(n w / W) or ceil(n w / W) times."""
    rng = np.random.default_rng(1)
    w = rng.exponential(1.0, 40)
    for u0 in (0.0, 0.3, 0.999):
        k = O.systematic_draws(w, 500, u0)
        counts = np.bincount(k, minlength=len(w))
        exp = 500 * w / w.sum()
        assert np.all(counts >= np.floor(exp) - 1e-9) and np.all(counts <= np.ceil(exp) + 1e-9)
        assert np.all(np.diff(k) >= 0)


def test_phase_draw_equal_weights():
    for u in (0.0, 0.26, 0.5, 0.999):
        assert O.inverse_cdf_index(np.ones(16), u) == math.floor(u * 16)


def test_distance_draw_empty_template():
    """dh = hh = 0: the posterior is the prior, P(D' >= D) = 1 - (D / D_max)^3
    (the draw inverts the distribution of v = d0/D)."""
    for u in (0.01, 0.3, 0.8, 0.999):
        assert O.distance_posterior_draw(0.0, 0.0, 5000.0, 1.0, u) == pytest.approx(
            5000.0 * (1.0 - u) ** (1.0 / 3.0), rel=1e-9)


@pytest.mark.parametrize("dh,hh", [(2.0e4, 1.0e8), (3.0e3, 2.0e7), (-1.0e3, 4.0e6), (50.0, 1e4)])
def test_distance_draw_round_trip(dh, hh):
    """The drawn D puts mass u above it: checked with a 200000-point
    trapezoid rule in ln D over (D_max 1e-6, D_max] (no shared code)."""
    d_max, d0 = 5000.0, 1.0
    x = np.linspace(math.log(d_max * 1e-6), math.log(d_max), 200001)
    D = np.exp(x)
    lg = 3.0 * x + dh * d0 / D - 0.5 * hh * (d0 / D) ** 2     # D^2 dD = D^3 d(ln D)
    f = np.exp(lg - lg.max())
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(x))])
    for u in (0.05, 0.5, 0.95):
        Ds = O.distance_posterior_draw(dh, hh, d_max, d0, u)
        assert 1.0 - np.interp(math.log(Ds), x, cum) / cum[-1] == pytest.approx(u, abs=2e-6)
