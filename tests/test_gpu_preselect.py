"""Intrinsic pre-selection on the GPU (dotpe_preselect) against the oracle
(Sec. IV D; App. B eqs. dh_itop, x_ML, single_det_ML): every detector's grid
maximum per row, the incoherent sums and the selection, on ragged row ranges
(not multiples of the 32-row blocks), with higher modes and the (2,2) mode
alone, an edge-on row, and a noise-free injection on the grid."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import workload as W

pytestmark = pytest.mark.gpu


def _tol(v):
    # FP16x2 operands (22 significant bits) with FP32 accumulation: the
    # projections carry ~1e-6 relative error, lnL^ML twice that
    return 1e-3 + 4e-6 * np.abs(v)


def _arrival(wl, ext1):
    la, lo = ext1["lat"], ext1["lon"]
    n = np.array([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)])
    return ext1["t_geo"] - wl.det_r @ n / 299792458.0


@pytest.fixture(scope="module")
def ctx():
    from paper_2507_16022_amd import dotpe
    c = dotpe.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("modes,prec", [(W.MODES_HM, "fp16x2"), (W.MODES_22, "fp16x2"),
                                        (W.MODES_HM, "bf16x2")])
def test_preselect_vs_oracle(ctx, modes, prec):
    wl = W.make_workload(21, n_int=230, n_ext=4, n_bins=128, modes=modes, dets="HLV", n_phi=16,
                         snr=25.0, mc_range=(8.0, 40.0), q_range=(0.2, 1.0), chi_range=(-0.5, 0.5))
    rng = np.random.default_rng(4)
    ci = rng.uniform(-1.0, 1.0, wl.n_int)
    ci[7] = 0.0                                   # edge-on: the 2x2 form is singular for (2,2)
    n_t, dt = 64, 5e-4
    t0 = _arrival(wl, wl.meta["inj_ext"]) - 0.5 * n_t * dt
    start, count = 37, 181                        # a range that straddles 32-row blocks
    bank = ctx.load_bank(wl.h, wl.modes, wl.f, precision=prec)
    r = ctx.preselect(bank, wl.d, wl.w, t0, dt, n_t, ci[start:start + count], wl.n_phi,
                      sub_start=start, sub_count=count, delta_lnl=20.0)
    bank.close()
    rows = np.arange(start, start + count)
    lnl, per = O.incoherent_ml(wl.h[rows], wl.modes, ci[rows], wl.f, wl.d, wl.w, t0, dt, n_t,
                               wl.n_phi)
    err = np.abs(r["lnl_det"] - per)
    print(f"pre-selection {prec} {len(modes)} modes: max |d lnL^ML_k| {err.max():.2e} "
          f"(values up to {per.max():.1f}); {r['n_selected']} of {count} rows kept; "
          f"{r['t_ms']:.2f} ms", flush=True)
    if prec == "bf16x2":
        # 16 significant bits: checked at its own, looser scale
        assert np.all(err <= 1e-2 + 1e-3 * np.abs(per))
        return
    assert np.all(err <= _tol(per))
    assert np.all(np.abs(r["lnl_inco"] - lnl) <= _tol(lnl) * 3)
    assert r["lnl_max"] == pytest.approx(lnl.max(), abs=float(_tol(lnl.max())) * 3)
    # the selection: every row clearly inside is kept, every row clearly out is not
    thr = lnl.max() - 20.0
    sel = set(r["selected"].tolist())
    assert all(start + q in sel for q in np.flatnonzero(lnl >= thr + 0.01))
    assert not any(start + q in sel for q in np.flatnonzero(lnl < thr - 0.01))
    assert list(r["selected"]) == sorted(r["selected"])


def test_preselect_noise_free_injection(ctx):
    """A bank row injected without noise at a grid time and phase: each
    detector's maximum is (d_k|d_k)/2 (the fit reproduces the data)."""
    wl = W.make_workload(23, n_int=40, n_ext=4, n_bins=128, modes=W.MODES_HM, dets="HLV",
                         n_phi=8, snr=20.0, mc_range=(8.0, 40.0), q_range=(0.2, 1.0),
                         chi_range=(-0.5, 0.5), noise_on=False)
    net = W.network("HLV")
    ext1 = {k: v[0] for k, v in W.draw_extrinsic(np.random.default_rng(2), 1).items()}
    ext1["cos_iota"] = 0.5
    row, o_star = 13, 5
    d = W.simulate_strain(wl.h[row], wl.modes, wl.f, net, ext1, 2 * np.pi * o_star / wl.n_phi, 300.0)
    n_t, dt, j_star = 32, 4e-4, 11
    t0 = _arrival(wl, ext1) - j_star * dt
    ci = np.full(wl.n_int, 0.5)
    bank = ctx.load_bank(wl.h, wl.modes, wl.f, precision="fp16x2")
    r = ctx.preselect(bank, d, wl.w, t0, dt, n_t, ci, wl.n_phi)
    bank.close()
    half = 0.5 * np.sum(wl.w * np.abs(d) ** 2, axis=1)
    print(f"noise-free injection: {r['lnl_det'][row]} vs {half}", flush=True)
    assert np.all(np.abs(r["lnl_det"][row] - half) <= _tol(half))
    assert r["lnl_inco"][row] == pytest.approx(half.sum(), abs=float(_tol(half.sum())) * 3)
    assert np.argmax(r["lnl_inco"]) == row and row in r["selected"]


def test_preselect_rejects(ctx):
    from paper_2507_16022_amd import dotpe
    wl = W.config_tiny(seed=3, n_int=40, n_ext=4)
    ci = np.zeros(wl.n_int)
    bank = ctx.load_bank(wl.h, wl.modes, wl.f, precision="fp16x2")
    t0 = np.zeros(2)
    with pytest.raises(dotpe.DotpeError):
        ctx.preselect(bank, wl.d, wl.w, t0, 1e-3, 48, ci, 8)          # n_t not a multiple of 32
    with pytest.raises(dotpe.DotpeError):
        ctx.preselect(bank, wl.d, wl.w, t0, 1e-3, 32, ci + 2.0, 8)    # |cos iota| > 1
    bank.close()
    b64 = ctx.load_bank(wl.h, wl.modes, wl.f, precision="fp64")
    with pytest.raises(dotpe.DotpeError):
        ctx.preselect(b64, wl.d, wl.w, t0, 1e-3, 32, ci, 8)           # FP64 bank
    b64.close()
