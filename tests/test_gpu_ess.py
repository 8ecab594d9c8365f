"""Effective sample sizes of the evidence pass (Sec. III B eq. n_effective;
Sec. V A eqs. posterior_element, int_ess, ext_ess) against the oracle: over
triples, intrinsic samples (row sums), extrinsic samples (column sums) and
pairs, for the FP64 and FP16x2 paths, without a cut and with one (the cut
pairs' mass is within the certificate, far below the tolerance)."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import workload as W

pytestmark = pytest.mark.gpu

KEYS = ("n_eff", "n_eff_int", "n_eff_ext", "n_eff_pairs")


@pytest.fixture(scope="module")
def ctx():
    from paper_2507_16022_amd import dotpe
    c = dotpe.Context(0)
    yield c
    c.close()


def _run(ctx, wl, prec, cut):
    bank = ctx.load_bank(wl.h, wl.modes, wl.f, wl.ln_w_int, precision=prec)
    ev = ctx.set_event(bank, d=wl.d, w=wl.w, det_r=wl.det_r, det_D=wl.det_D, ext=wl.ext,
                       n_phi=wl.n_phi, ln_w_ext=wl.ln_w_ext, d_max=wl.d_max, d0=wl.d0,
                       cut_delta=cut)
    r = ev.evidence()
    ev.close()
    bank.close()
    return r


@pytest.mark.parametrize("cfg", ["tiny", "hm"])
def test_effective_sizes_vs_oracle(ctx, cfg):
    # quiet events, so that the posterior spreads over many pairs and the
    # four sizes differ from each other
    if cfg == "tiny":
        wl = W.config_tiny(seed=5, snr=4.0).subset(rows=np.arange(150), cols=np.arange(200))
    else:
        wl = W.config_production(seed=6, snr=6.0, n_int=90, n_ext=130)
    ref = O.effective_sizes(O.posterior_weights(wl))
    assert ref["n_eff"] > 30 and ref["n_eff_int"] > 4 and ref["n_eff_ext"] > 6
    for prec, cut, rel in (("fp64", 0.0, 1e-6), ("fp16x2", 0.0, 2e-4), ("fp16x2", 15.0, 5e-4)):
        r = _run(ctx, wl, prec, cut)
        msg = ", ".join(f"{k} {r[k]:.6g}/{ref[k]:.6g}" for k in KEYS)
        print(f"{cfg} {prec} cut {cut}: {msg}", flush=True)
        for k in KEYS:
            assert r[k] == pytest.approx(ref[k], rel=rel), (prec, cut, k)
