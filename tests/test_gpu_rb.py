"""The paper's own layout and relative binning on the GPU against the
oracle: relative-binning weights from full-resolution data (App. A eqs.
dh_weights, hh_weights), per-pair likelihoods and the evidence with those
weights (eqs. d_h, h_h), and banks in the (m, p) layout (Sec. IV A eq. h_k:
real antenna patterns, the inclination in the bank) with three detectors,
for the FP64 and FP16x2 paths."""
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


def _pols_and_m(wl, layout):
    if layout == "mp":
        return [p for _, p in wl.modes], np.array([m for m, _ in wl.modes], dtype=np.float64)
    return None, np.array([m for _, m in wl.modes], dtype=np.float64)


def _oracle_pairs(wl, layout, Wdh, Whh):
    pols, mm = _pols_and_m(wl, layout)
    R = O.response_mp(wl.det_D, pols, wl.ext) if layout == "mp" else O.response(wl.det_D, wl.modes, wl.ext)
    t = O.arrival_times(wl.det_r, wl.ext["lat"], wl.ext["lon"], wl.ext["t_geo"])
    return O.eval_pairs_general(wl.h, mm, R, t, wl.f, wl.n_phi, Wdh, Whh, wl.ln_w_int, wl.ln_w_ext,
                                wl.d_max, wl.d0)


def _event(ctx, wl, prec, layout, **kw):
    bank = ctx.load_bank(wl.h, wl.modes, wl.f, wl.ln_w_int, precision=prec, layout=layout)
    ev = ctx.set_event(bank, d=kw.pop("d", wl.d), w=kw.pop("w", wl.w), det_r=wl.det_r, det_D=wl.det_D,
                       ext=wl.ext, n_phi=wl.n_phi, ln_w_ext=wl.ln_w_ext, d_max=wl.d_max, d0=wl.d0,
                       **kw)
    return bank, ev


@pytest.mark.parametrize("layout", ["lm", "mp"])
def test_rb_weights_vs_oracle(ctx, layout):
    ev = W.make_rb_event(11, 4, 4, 64, 5000, layout=layout)
    g_dh, g_hh, g_dd = ctx.rb_weights(ev.f_full, ev.d_full, ev.w_full, ev.h0, ev.node_idx, ev.t0)
    r_dh, r_hh, r_dd = O.rb_weights(ev.f_full, ev.d_full, ev.w_full, ev.h0, ev.node_idx, ev.t0)
    e_dh = np.max(np.abs(g_dh - r_dh)) / np.max(np.abs(r_dh))
    e_hh = np.max(np.abs(g_hh - r_hh)) / np.max(np.abs(r_hh))
    print(f"rb weights {layout}: rel err W_dh {e_dh:.2e}, W_hh {e_hh:.2e}, dd {g_dd / r_dd - 1:.1e}",
          flush=True)
    assert e_dh <= 1e-11 and e_hh <= 1e-11
    assert g_dd == pytest.approx(r_dd, rel=1e-12)


@pytest.mark.parametrize("layout", ["lm", "mp"])
def test_rb_pairs_and_evidence_vs_oracle(ctx, layout):
    """Each side builds its own weights from the same full-resolution inputs."""
    rbe = W.make_rb_event(12, 50, 70, 64, 5000, layout=layout, snr=25.0)
    wl = rbe.wl
    g_dh, g_hh, g_dd = ctx.rb_weights(rbe.f_full, rbe.d_full, rbe.w_full, rbe.h0, rbe.node_idx, rbe.t0)
    r_dh, r_hh, r_dd = O.rb_weights(rbe.f_full, rbe.d_full, rbe.w_full, rbe.h0, rbe.node_idx, rbe.t0)
    ref = _oracle_pairs(wl, layout, r_dh, r_hh)
    ln_z = O.evidence_general(ref, wl.n_int, wl.n_ext)
    for prec, tol in (("fp64", 1e-6), ("fp16x2", 1e-3)):
        bank, ev = _event(ctx, wl, prec, layout, d=None, w=None, w_dh=g_dh, w_hh=g_hh, dd=g_dd)
        out = ev.eval_lnl(ml=True)
        r = ev.evidence()
        ev.close()
        bank.close()
        err = np.max(np.abs(out["lnl"] - ref["lnl"]))
        print(f"rb {layout} {prec}: max lnL^ML {ref['ml_max'].max():.2f}, max |d lnLbar| {err:.2e}, "
              f"ln Z {r['ln_z']:.8f} vs {ln_z:.8f}", flush=True)
        assert err <= tol
        assert abs(r["ln_z"] - ln_z) <= tol
        assert r["dd"] == pytest.approx(r_dd, rel=1e-12)
        assert r["max_lnl_ml"] == pytest.approx(float(ref["ml_max"].max()), rel=1e-6, abs=tol)


def test_mp_layout_plain_bins_vs_oracle(ctx):
    """An (m, p) bank (8 channels, 4 m values) on the plain bins of a three-detector
    event: per pair and the evidence, with and without the cut."""
    wl0 = W.config_production(seed=13, n_int=48, n_ext=70, snr=20.0, random_weights=True)
    rng = np.random.default_rng(2)
    h, chans = W.waveform_mp(wl0.f, wl0.meta["mc"], wl0.meta["q"], wl0.meta["chi"],
                             rng.uniform(-0.95, 0.95, wl0.n_int), wl0.modes)
    wl = W.Workload(chans, wl0.f, h, wl0.ln_w_int, wl0.det_r, wl0.det_D, wl0.d, wl0.w, wl0.ext,
                    wl0.ln_w_ext, wl0.n_phi, wl0.d_max, wl0.d0)
    K, C, B = wl.d.shape[0], h.shape[1], wl.d.shape[1]
    Wdh = np.broadcast_to((wl.w * wl.d)[:, None, :], (K, C, B))
    Whh = np.broadcast_to(wl.w[:, None, None, :], (K, C, C, B)).astype(np.complex128)
    ref = _oracle_pairs(wl, "mp", Wdh, Whh)
    ln_z = O.evidence_general(ref, wl.n_int, wl.n_ext)
    for prec, tol in (("fp64", 1e-6), ("fp16x2", 1e-3)):
        for cut in (0.0, 30.0):
            bank, ev = _event(ctx, wl, prec, "mp", cut_delta=cut)
            out = ev.eval_lnl()
            r = ev.evidence()
            ev.close()
            bank.close()
            err = np.max(np.abs(out["lnl"] - ref["lnl"]))
            print(f"mp {prec} cut {cut}: max lnL^ML {ref['ml_max'].max():.2f}, max |d lnLbar| "
                  f"{err:.2e}, ln Z {r['ln_z']:.8f} (upper {r['ln_z_upper']:.8f}) vs {ln_z:.8f}, "
                  f"bounded {r['n_pairs_bounded']}", flush=True)
            assert err <= tol
            assert r["ln_z"] <= ln_z + tol and ln_z <= r["ln_z_upper"] + tol
            assert abs(r["ln_z"] - ln_z) <= tol + (r["ln_z_upper"] - r["ln_z"])


def _mp_workload(seed, n_int, n_ext, snr=20.0):
    wl0 = W.config_production(seed=seed, n_int=n_int, n_ext=n_ext, snr=snr, random_weights=True)
    rng = np.random.default_rng(seed + 100)
    h, chans = W.waveform_mp(wl0.f, wl0.meta["mc"], wl0.meta["q"], wl0.meta["chi"],
                             rng.uniform(-0.95, 0.95, wl0.n_int), wl0.modes)
    return W.Workload(chans, wl0.f, h, wl0.ln_w_int, wl0.det_r, wl0.det_D, wl0.d, wl0.w, wl0.ext,
                      wl0.ln_w_ext, wl0.n_phi, wl0.d_max, wl0.d0)


def test_mp_layout_bound_pass_certified(ctx):
    """Every pair's bound from the bound pass of an (m, p) bank (folded (h|h)
    sums) is above the bound formed from the oracle's exact phase
    coefficients."""
    from test_gpu_bound import _exact_bound
    wl = _mp_workload(14, 60, 80)
    K, C, B = wl.d.shape[0], wl.h.shape[1], wl.d.shape[1]
    Wdh = np.broadcast_to((wl.w * wl.d)[:, None, :], (K, C, B))
    Whh = np.broadcast_to(wl.w[:, None, None, :], (K, C, C, B)).astype(np.complex128)
    ref = _oracle_pairs(wl, "mp", Wdh, Whh)
    ex = _exact_bound(ref["dh"], ref["hh"], [m for m, _ in wl.modes])
    bank, ev = _event(ctx, wl, "fp16x2", "mp")
    bd = ev.bound()
    ev.close()
    bank.close()
    fin = np.isfinite(ex)
    for name, b in (("whole rows", bd[0]), ("per group", bd[1])):
        b = b.astype(np.float64)
        top = fin & (ref["ml_max"] >= ref["ml_max"].max() - 40.0)
        print(f"mp bound, margin of {name}: max excess within 40 of the max "
              f"{np.max((b - ex)[top] / ex[top]):.3g}", flush=True)
        assert np.all(b >= 1.0008 * np.where(fin, ex, 0.0))
        assert np.all(b >= 1.0005 * ref["ml_max"])


def test_mp_layout_large_event_cut(ctx):
    """An (m, p) event large enough for the bound pass (8192 x 4096): the cut
    evidence within its certificate of the uncut one, and the best pairs'
    ln p against the oracle."""
    wl = _mp_workload(15, 8192, 4096, snr=20.0)
    res = {}
    for cut in (0.0, 30.0):
        bank, ev = _event(ctx, wl, "fp16x2", "mp", cut_delta=cut, top_k=16)
        res[cut] = ev.evidence()
        ev.close()
        bank.close()
    a, b = res[30.0], res[0.0]
    print(f"mp large: ln Z cut {a['ln_z']:.8f} (upper {a['ln_z_upper']:.8f}, bounded "
          f"{a['n_pairs_bounded']}, listed tiles {a['n_tiles_listed']}) vs uncut {b['ln_z']:.8f}",
          flush=True)
    assert a["n_pairs_bounded"] > 0.99 * a["n_pairs"]
    # the survivors are evaluated in FP64 from the split operands, the uncut
    # pass's pairs by the split products: the two agree to the FP16x2 tolerance
    assert a["ln_z_upper"] - a["ln_z"] <= 1e-4
    assert abs(a["ln_z"] - b["ln_z"]) <= 1e-3
    rows, cols = a["topk_i"][:16], a["topk_e"][:16]
    sub = W.Workload(wl.modes, wl.f, wl.h[rows], wl.ln_w_int[rows], wl.det_r, wl.det_D, wl.d, wl.w,
                     {k: v[cols] for k, v in wl.ext.items()}, wl.ln_w_ext[cols], wl.n_phi, wl.d_max,
                     wl.d0)
    K, C, B = wl.d.shape[0], wl.h.shape[1], wl.d.shape[1]
    Wdh = np.broadcast_to((wl.w * wl.d)[:, None, :], (K, C, B))
    Whh = np.broadcast_to(wl.w[:, None, None, :], (K, C, C, B)).astype(np.complex128)
    ref = _oracle_pairs(sub, "mp", Wdh, Whh)
    lnp = np.diag(ref["lnp"])
    err = np.max(np.abs(a["topk_lnp"][:16] - lnp))
    print(f"   top-16 vs oracle: max |d ln p| {err:.2e}", flush=True)
    assert err <= 1e-3
