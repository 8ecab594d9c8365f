"""Pins of the oracle's extrinsic-sample proposal (Sec. IV E; App. C): the
equal-area sky lattice, the flat-probability limit, the importance-sampling
identity, the geometry of a noise-free injection, and unbiasedness of the
weights by Monte Carlo."""
import math

import numpy as np

from oracle import oracle as O
from synth import workload as W


def test_fibonacci_sky_is_equal_area():
    lat, lon = O.fibonacci_sky(4096)
    n = O.sky_direction(lat, lon)
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0)
    # equal-area points: z uniform on (-1, 1), moments of the isotropic distribution
    assert np.allclose(np.sort(n[:, 2]), np.sort(1.0 - (2.0 * np.arange(4096) + 1.0) / 4096))
    assert np.max(np.abs(n.mean(0))) < 2e-3
    assert np.max(np.abs(n.T @ n / 4096 - np.eye(3) / 3)) < 2e-3


def _setup(beta=0.5, n_sky=512, n_tg=24, wide=False):
    wl = W.config_tiny(seed=21, snr=25.0, in_bank=True, noise_on=False)
    rows = np.array([0, 1, 2, 3])
    ci = np.full(len(rows), wl.ext["cos_iota"][0])
    n_t, dt = 96, 5e-4
    # detector grids around the injected arrival times (wide: the whole light-travel window)
    ext0 = {k: v[0] for k, v in wl.ext.items()}
    t_inj = O.arrival_times(wl.det_r, [ext0["lat"]], [ext0["lon"]], [ext0["t_geo"]])[0]
    t0 = (t_inj - 0.5 * n_t * dt) if not wide else np.full(len(t_inj), ext0["t_geo"] - 0.024)
    rho2 = O.arrival_time_series(wl.h[rows], wl.modes, ci, wl.f, wl.d, wl.w, t0, dt, n_t, 8)
    lat, lon = O.fibonacci_sky(n_sky)
    tg_lo, tg_hi = ext0["t_geo"] - 0.012, ext0["t_geo"] + 0.012
    lnW, lnZ = O.proposal_table(rho2, t0, dt, wl.det_r, lat, lon, tg_lo, tg_hi, n_tg, beta)
    return dict(wl=wl, rho2=rho2, lat=lat, lon=lon, lnW=lnW, lnZ=lnZ, tg=(tg_lo, tg_hi), t0=t0,
                dt=dt, n_t=n_t, t_inj=t_inj, ext0=ext0)


def test_flat_probabilities_give_equal_weights():
    s = _setup(beta=0.0, wide=True)
    P = np.exp(s["lnW"] - s["lnZ"][:, None, None])
    assert np.allclose(P.reshape(len(P), -1).sum(1), 1.0)
    supp = np.isfinite(s["lnW"][0])
    # beta = 0: every cell whose arrival times all fall on the grids is equally likely
    assert np.all(np.isfinite(s["lnW"]) == supp[None])
    assert np.allclose(P[:, supp], 1.0 / supp.sum())
    out = O.extrinsic_proposal(s["lnW"], s["lnZ"], s["lat"], s["lon"], *s["tg"], 64, 5)
    assert np.allclose(out["ln_w"], math.log(supp.sum() / supp.size))


def test_importance_identity_and_geometry():
    s = _setup()
    C, S, J = s["lnW"].shape
    P = np.exp(s["lnW"] - s["lnZ"][:, None, None]).reshape(C, -1)
    mix = P.mean(0)
    supp = mix > 0
    ln_w = -math.log(S * J) - np.log(mix[supp])
    # sum over cells of pi' w = the prior mass of the proposal's support
    assert abs(np.sum(mix[supp] * np.exp(ln_w)) - supp.sum() / (S * J)) < 1e-12
    # the injected row's most probable cell puts the signal at each detector
    # within a grid step of its true arrival time
    cell = int(np.argmax(P[0]))
    sidx, j = divmod(cell, J)
    tj = s["tg"][0] + (j + 0.5) * (s["tg"][1] - s["tg"][0]) / J
    n = O.sky_direction([s["lat"][sidx]], [s["lon"][sidx]])[0]
    t_k = tj - (s["wl"].det_r @ n) / O.C_SI
    assert np.max(np.abs(t_k - s["t_inj"])) <= 1.5 * s["dt"] + (s["tg"][1] - s["tg"][0]) / J


def test_weights_unbiased_by_monte_carlo():
    s = _setup(n_sky=256, n_tg=16)
    C, S, J = s["lnW"].shape
    out = O.extrinsic_proposal(s["lnW"], s["lnZ"], s["lat"], s["lon"], *s["tg"], 6000, 17)
    P = np.exp(s["lnW"] - s["lnZ"][:, None, None]).reshape(C, -1)
    supp = P.mean(0) > 0
    w = np.exp(out["ln_w"])
    target = supp.sum() / (S * J)
    # E_pi'[w] = the prior mass of the support; 6 standard errors
    assert abs(w.mean() - target) <= 6 * w.std() / math.sqrt(len(w)) + 1e-12
    # the prior parts are prior draws
    assert 0.0 <= out["psi"].min() and out["psi"].max() < math.pi
    assert -1.0 <= out["cos_iota"].min() and out["cos_iota"].max() < 1.0
    # stratified: draw q from component q mod C, whose support holds its cell
    for q in range(0, 6000, 97):
        assert P[q % C, out["cell"][q]] > 0
