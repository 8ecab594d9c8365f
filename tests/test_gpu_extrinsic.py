"""Extrinsic samples by importance sampling (dotpe_extrinsic_samples; Sec.
IV E, App. C) against the oracle: the same SplitMix64 uniforms, so the prior
parts (psi, cos iota) match exactly and the cells match where the oracle's
proposal does not put the draw within rounding of a cell boundary (the
arrival-time series come from the pre-selection's FP32 epilogue); weights,
the effective sample size of the weights and the support."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from synth import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2507_16022_amd import dotpe
    c = dotpe.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("cfg", ["tiny", "hm"])
def test_extrinsic_samples_vs_oracle(ctx, cfg):
    if cfg == "tiny":
        wl = W.config_tiny(seed=21, snr=25.0, in_bank=True, noise_on=False)
        n_phi, n_sky, n_tg = 8, 512, 24
    else:
        wl = W.config_production(seed=22, n_int=8, n_ext=4, snr=20.0, in_bank=True)
        n_phi, n_sky, n_tg = 16, 1024, 32
    rows = np.array([0, 1, 2, 3])
    ci = np.full(len(rows), wl.ext["cos_iota"][0])
    n_t, dt = 96, 5e-4
    ext0 = {k: v[0] for k, v in wl.ext.items()}
    t_inj = O.arrival_times(wl.det_r, [ext0["lat"]], [ext0["lon"]], [ext0["t_geo"]])[0]
    t0 = t_inj - 0.5 * n_t * dt
    tg_lo, tg_hi = ext0["t_geo"] - 0.012, ext0["t_geo"] + 0.012
    n_s, seed = 600, 77
    bank = ctx.load_bank(wl.h, wl.modes, wl.f, wl.ln_w_int, precision="fp16x2")
    g = ctx.extrinsic_samples(bank, wl.d, wl.w, wl.det_r, t0, dt, n_t, rows, ci, n_phi, n_sky, n_tg,
                              tg_lo, tg_hi, n_s, seed=seed)
    bank.close()
    rho2 = O.arrival_time_series(wl.h[rows], wl.modes, ci, wl.f, wl.d, wl.w, t0, dt, n_t, n_phi)
    lat, lon = O.fibonacci_sky(n_sky)
    lnW, lnZ = O.proposal_table(rho2, t0, dt, wl.det_r, lat, lon, tg_lo, tg_hi, n_tg, 0.5)
    ref = O.extrinsic_proposal(lnW, lnZ, lat, lon, tg_lo, tg_hi, n_s, seed)
    C = len(rows)
    P = np.exp(lnW - lnZ[:, None, None]).reshape(C, -1)
    dtg = (tg_hi - tg_lo) / n_tg
    # the GPU's cells from its outputs
    n_g = O.sky_direction(g["lat"], g["lon"])
    n_l = O.sky_direction(lat, lon)
    s_g = np.argmax(n_g @ n_l.T, axis=1)
    assert np.max(np.abs(n_l[s_g] - n_g)) < 1e-9
    j_g = np.floor((g["t_geo"] - tg_lo) / dtg).astype(np.int64)
    cell_g = s_g * n_tg + j_g
    same = cell_g == ref["cell"]
    for q in np.flatnonzero(~same):
        cum = np.cumsum(P[q % C])
        u = O.splitmix64_uniform(seed, 4 * q)
        k = cell_g[q]
        lo = cum[k - 1] if k > 0 else 0.0
        assert lo - 1e-2 <= u <= cum[k] + 1e-2, q
    assert np.allclose(g["psi"], ref["psi"], rtol=1e-14, atol=0)
    assert np.allclose(g["cos_iota"], ref["cos_iota"], rtol=0, atol=1e-14)
    assert np.allclose(g["t_geo"][same], ref["t_geo"][same], rtol=0, atol=1e-12)
    assert np.max(np.abs(g["ln_w"][same] - ref["ln_w"][same])) < 2e-2
    def n_eff(lw):
        w = np.exp(lw - lw.max())
        return w.sum() ** 2 / (w ** 2).sum()

    supp = np.mean(P.mean(0) > 0)
    print(f"{cfg}: {same.mean():.3f} of the cells as the oracle draws them; N_eff prior "
          f"{g['n_eff_prior']:.1f} (oracle draws {n_eff(ref['ln_w']):.1f}; on the common cells "
          f"{n_eff(g['ln_w'][same]):.1f} vs {n_eff(ref['ln_w'][same]):.1f}); support "
          f"{g['support']:.4f} vs {supp:.4f}; {g['t_ms']:.2f} ms", flush=True)
    assert same.mean() >= 0.9
    # the reported size is that of the returned weights; where the draws agree
    # it is the oracle's (a single draw in a cell of tiny probability, which
    # rounding may send to its neighbour, moves the size of the whole set)
    assert g["n_eff_prior"] == pytest.approx(n_eff(g["ln_w"]), rel=1e-9)
    assert n_eff(g["ln_w"][same]) == pytest.approx(n_eff(ref["ln_w"][same]), rel=0.05)
    assert g["support"] == pytest.approx(supp, abs=1e-2)
    assert np.isfinite(g["ln_w"]).all()
