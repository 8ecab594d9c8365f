"""Pins of the oracle's effective sample sizes (Sec. III B eq. n_effective;
Sec. V A eqs. posterior_element, int_ess, ext_ess): equal weights, a single
weight, weights that factorise (closed forms), bounds, and the consistency
of the per-triple weights with the per-pair likelihood."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from synth import workload as W


def test_equal_weights_count_everything():
    lnp = np.full((5, 7, 4), -3.0)
    r = O.effective_sizes(lnp)
    assert r["n_eff"] == pytest.approx(5 * 7 * 4, rel=1e-12)
    assert r["n_eff_int"] == pytest.approx(5, rel=1e-12)
    assert r["n_eff_ext"] == pytest.approx(7, rel=1e-12)
    assert r["n_eff_pairs"] == pytest.approx(35, rel=1e-12)


def test_single_weight_is_one():
    lnp = np.full((3, 4, 5), -np.inf)
    lnp[1, 2, 3] = 7.0
    r = O.effective_sizes(lnp)
    for k in ("n_eff", "n_eff_int", "n_eff_ext", "n_eff_pairs"):
        assert r[k] == pytest.approx(1.0, rel=1e-12)


def test_factorised_weights_closed_form():
    """p_ieo = a_i b_e c_o: every sum factorises, so N_eff,int = (sum a)^2 /
    sum a^2, N_eff,ext likewise with b, and N_eff over triples is the
    product of the three ratios."""
    rng = np.random.default_rng(0)
    a, b, c = rng.uniform(0.1, 3.0, 6), rng.uniform(0.1, 3.0, 9), rng.uniform(0.1, 3.0, 4)
    lnp = np.log(a)[:, None, None] + np.log(b)[None, :, None] + np.log(c)[None, None, :]
    r = O.effective_sizes(lnp)
    ra, rb, rc = (a.sum() ** 2 / (a * a).sum(), b.sum() ** 2 / (b * b).sum(),
                  c.sum() ** 2 / (c * c).sum())
    assert r["n_eff_int"] == pytest.approx(ra, rel=1e-12)
    assert r["n_eff_ext"] == pytest.approx(rb, rel=1e-12)
    assert r["n_eff"] == pytest.approx(ra * rb * rc, rel=1e-12)
    assert r["n_eff_pairs"] == pytest.approx(ra * rb, rel=1e-12)


def test_bounds_and_phase_sum():
    """1 <= N_eff <= N for any weights; and the triple weights of a
    workload sum over the phases to the pair weights of eq. (Z_sum)."""
    wl = W.config_tiny(seed=2, n_int=6, n_ext=10)
    lnp3 = O.posterior_weights(wl)
    r = O.effective_sizes(lnp3)
    assert 1.0 <= r["n_eff"] <= lnp3.size
    assert 1.0 <= r["n_eff_int"] <= lnp3.shape[0]
    assert 1.0 <= r["n_eff_ext"] <= lnp3.shape[1]
    lnl = O.eval_lnl(wl)["lnl"]
    ev = O.evidence_from_lnl(lnl, wl.ln_w_int, wl.ln_w_ext)
    assert np.allclose(O._lse(lnp3, axis=2), ev["lnp"], rtol=0, atol=1e-10)
    # the pair-level ratio is eq. (n_effective) over the pairs
    assert r["n_eff_pairs"] == pytest.approx(ev["n_eff"], rel=1e-10)
