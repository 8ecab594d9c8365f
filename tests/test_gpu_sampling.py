"""Posterior samples (dotpe_sample_posterior; Sec. III B resampling by the
probabilistic weights, Sec. V B N_s = N_eff / 2) against the oracle: the
same systematic draws over the pairs in the library's enumeration order
(64 x 64 tiles in row-major order, pairs row-major within a tile), the same
SplitMix64 uniforms for the phase and distance draws.  Where a draw falls
within rounding of a boundary between two pairs or phases either side is
correct, so the check is that the chosen one brackets the draw."""
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


def _tile_order(n_i, n_e, tm=64, tn=64):
    order = []
    for a in range(0, n_i, tm):
        for b in range(0, n_e, tn):
            for i in range(a, min(a + tm, n_i)):
                for e in range(b, min(b + tn, n_e)):
                    order.append((i, e))
    return np.array(order)


def _brackets(weights, k, u, tol):
    cum = np.cumsum(weights)
    lo = cum[k - 1] if k > 0 else 0.0
    return lo - tol * cum[-1] <= u * cum[-1] <= cum[k] + tol * cum[-1]


@pytest.mark.parametrize("cfg", ["tiny", "hm"])
def test_samples_vs_oracle(ctx, cfg):
    if cfg == "tiny":
        wl = W.config_tiny(seed=5, snr=4.0).subset(rows=np.arange(150), cols=np.arange(200))
    else:
        wl = W.config_production(seed=6, snr=6.0, n_int=90, n_ext=130)
    n_s, u0, seed = 300, 0.37, 99
    bank = ctx.load_bank(wl.h, wl.modes, wl.f, wl.ln_w_int, precision="fp16x2")
    ev = ctx.set_event(bank, d=wl.d, w=wl.w, det_r=wl.det_r, det_D=wl.det_D, ext=wl.ext,
                       n_phi=wl.n_phi, ln_w_ext=wl.ln_w_ext, d_max=wl.d_max, d0=wl.d0)
    r = ev.evidence()
    smp = ev.sample_posterior(n_samples=n_s, u0=u0, seed=seed)
    dflt = ev.sample_posterior()
    ev.close()
    bank.close()
    assert len(dflt["i"]) == max(1, math.floor(r["n_eff"] / 2))
    ref = O.eval_pairs_block(wl, np.arange(wl.n_int), return_triples=True, return_phase=True)
    lnp3 = (wl.ln_w_int[:, None, None] + wl.ln_w_ext[None, :, None] + ref["lnl_phase"]
            - math.log(wl.n_phi))
    lnp = O._lse(lnp3, axis=2)
    order = _tile_order(wl.n_int, wl.n_ext)
    w = np.exp(lnp[order[:, 0], order[:, 1]] - lnp.max())
    expect = O.systematic_draws(w, n_s, u0)
    pos = {tuple(p): q for q, p in enumerate(order)}
    same_pair = 0
    same_phase = 0
    for s in range(n_s):
        i, e, o = int(smp["i"][s]), int(smp["e"][s]), int(smp["o"][s])
        k = pos[(i, e)]
        if k == expect[s]:
            same_pair += 1
        else:
            assert _brackets(w, k, (s + u0) / n_s, 1e-5), s
        assert smp["ln_p_pair"][s] == pytest.approx(lnp[i, e], abs=1e-3)
        assert smp["ln_p_triple"][s] == pytest.approx(lnp3[i, e, o], abs=1e-3)
        wo = np.exp(ref["lnl_phase"][i, e] - ref["lnl_phase"][i, e].max())
        u_phi = O.splitmix64_uniform(seed, 2 * s)
        if O.inverse_cdf_index(wo, u_phi) == o:
            same_phase += 1
        else:
            assert _brackets(wo, o, u_phi, 1e-5), s
        d_ref = O.distance_posterior_draw(ref["dh"][i, e, o], ref["hh"][i, e, o], wl.d_max, wl.d0,
                                          O.splitmix64_uniform(seed, 2 * s + 1))
        assert smp["distance"][s] == pytest.approx(d_ref, rel=1e-3), s
    print(f"{cfg}: N_eff {r['n_eff']:.1f}; {same_pair}/{n_s} pairs and {same_phase}/{n_s} phases "
          f"as the oracle draws them", flush=True)
    assert same_pair >= 0.95 * n_s and same_phase >= 0.95 * n_s
