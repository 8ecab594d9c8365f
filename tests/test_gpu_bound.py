"""The bound pass of the evidence (128 x 128 tiles that only bound every
pair, tiles with survivors evaluated by the second, batched pass) against
the fused kernel's own bound-then-evaluate epilogue and against the FP64
path, at shapes with ragged edges in both directions, with a contiguous
bank range and with scattered rows."""
import numpy as np
import pytest

from synth import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2507_16022_amd import dotpe
    wl = W.config_production(seed=51, n_int=70001, n_ext=3001, snr=30.0, with_bank=False,
                             random_weights=True)
    h = W.bank_on_device(torch, wl.meta["mc"], wl.meta["q"], wl.meta["chi"], wl.f, wl.modes)
    lw = torch.as_tensor(np.random.default_rng(5).normal(0.0, 0.5, wl.meta["mc"].shape[0])).cuda()
    ctx = dotpe.Context(0)
    banks = {p: ctx.load_bank(h, wl.modes, wl.f, lw, precision=p) for p in ("fp16x2", "bf16x2", "fp64")}
    yield dotpe, wl, ctx, banks
    for b in banks.values():
        b.close()
    ctx.close()


def _run(ctx, bank, wl, **kw):
    ev = ctx.set_event(bank, d=wl.d, w=wl.w, det_r=wl.det_r, det_D=wl.det_D, ext=wl.ext,
                       n_phi=wl.n_phi, ln_w_ext=wl.ln_w_ext, d_max=wl.d_max, d0=wl.d0, top_k=48,
                       topk_window=30.0, **kw)
    r = ev.evidence()
    ev.close()
    return r


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x2"])
@pytest.mark.parametrize("cut", [40.0, 12.0, 0.0])
@pytest.mark.parametrize("rows", ["range", "scattered"])
def test_bound_pass_agrees(env, prec, cut, rows):
    dotpe, wl, ctx, banks = env
    n = wl.meta["mc"].shape[0]
    kw = dict(cut_delta=cut)
    if rows == "scattered":
        kw["sub_idx"] = np.random.default_rng(3).permutation(n)[: n - 1234].astype(np.int64)
        kw["n_norm"] = float(n)
    a = _run(ctx, banks[prec], wl, **kw)
    b = _run(ctx, banks[prec], wl, flags=dotpe.FLAG_NO_BOUND_PASS, **kw)
    print(f"bound pass {prec} cut {cut} {rows}: ln Z {a['ln_z']:.10f} vs {b['ln_z']:.10f}; "
          f"rerun tiles {a['n_tiles_rerun']}, listed {a['n_tiles_listed']}; main {a['t_main_ms']:.2f} ms "
          f"vs {b['t_main_ms']:.2f} ms; whole {a['t_fused_ms']:.2f} ms vs {b['t_fused_ms']:.2f} ms",
          flush=True)
    assert a["n_pairs"] == b["n_pairs"]
    assert a["n_tiles_rerun"] + a["n_tiles_listed"] > 0
    # the bound pass bounds from the hi parts alone plus a margin, so it
    # leaves a few more pairs to evaluate than the fused kernel's bound from
    # the full accumulators; the survivors' inner products are summed in
    # FP64 on one route and in FP32 on the matrix cores on the other, so the
    # rest agrees to rounding
    print(f"   bounded pairs {a['n_pairs_bounded']} vs {b['n_pairs_bounded']}; triples "
          f"marginalised {a['n_triples_marg']} vs {b['n_triples_marg']}", flush=True)
    assert 0.99 * b["n_pairs_bounded"] <= a["n_pairs_bounded"] <= b["n_pairs_bounded"] + 16
    assert a["n_triples_marg"] >= (1 - 1e-3) * b["n_triples_marg"] - 2
    for k in ("ln_z", "ln_z_upper", "ln_sum_p2", "max_lnl_ml", "max_ln_p", "ln_sum_p2_triples",
              "ln_sum_row2", "ln_sum_col2"):
        assert abs(a[k] - b[k]) <= 1e-3, k
    assert a["topk_count"] == b["topk_count"] and a["topk_count"] > 0
    assert np.max(np.abs(a["topk_lnp"] - b["topk_lnp"])) <= 1e-3
    # (with a cut narrower than the top-k window, cut pairs may lie in the window)
    if cut >= 30.0:
        assert a["topk_exact"] == b["topk_exact"] == 1
    assert a["ln_z_upper"] - a["ln_z"] <= 1e-4
    if prec == "fp16x2":
        c = _run(ctx, banks["fp64"], wl, **kw)
        print(f"   fp64 path: ln Z {c['ln_z']:.10f}; top-16 |d ln p| bound route "
              f"{np.max(np.abs(a['topk_lnp'][:16] - c['topk_lnp'][:16])):.2e}, fused route "
              f"{np.max(np.abs(b['topk_lnp'][:16] - c['topk_lnp'][:16])):.2e}", flush=True)
        for r in (a, b):
            assert abs(r["ln_z"] - c["ln_z"]) <= 1e-3
            assert np.max(np.abs(r["topk_lnp"][:16] - c["topk_lnp"][:16])) <= 1e-3


def _exact_bound(dh, hh, ms):
    """The bound from exact phase coefficients: dh_o = Re sum_g X_g e^(i m_g phi_o)
    and hh_o = S0 + 2 Re sum_d S_d e^(-i d phi_o) are trigonometric sums of
    degree < N_phi / 2, so their grid transforms give |X_g|, S0 and |S_d|;
    then U = sum_g |X_g|, lo = S0 - 2 sum_d |S_d| and U^2 / (2 lo)."""
    n = dh.shape[-1]
    phi = 2.0 * np.pi * np.arange(n) / n
    U = sum(np.abs(2.0 / n * np.sum(dh * np.exp(-1j * m * phi), axis=-1)) for m in sorted(set(ms)))
    S0 = np.mean(hh, axis=-1)
    lo = S0 - 2.0 * sum(np.abs(np.mean(hh * np.exp(1j * d * phi), axis=-1))
                        for d in range(1, max(ms) - min(ms) + 1))
    with np.errstate(divide="ignore"):
        return np.where(lo > 0, U * U / (2.0 * np.where(lo > 0, lo, 1.0)), np.inf)


@pytest.mark.parametrize("cfg,snr", [("tiny", 20.0), ("tiny", 50.0), ("hm", 20.0), ("hm", 50.0)])
def test_bound_certified_per_pair(cfg, snr):
    """Every pair's bound from the bound pass (hi parts of the split operands
    plus the Cauchy-Schwarz margin) against the same bound formed from the
    oracle's exact inner products: never below it by more than the bound's
    own 0.1% factor allows (so never below the pair's largest lnL^ML, eq.
    bestfit_lnl), and, where the cut decides, not far above it; at ragged
    shapes, for both split precisions."""
    from oracle import oracle as O
    from paper_2507_16022_amd import dotpe
    if cfg == "tiny":
        wl = W.config_tiny(seed=8, snr=snr).subset(rows=np.arange(150), cols=np.arange(200))
    else:
        wl = W.config_production(seed=9, snr=snr, n_int=140, n_ext=190)
    ref = O.eval_pairs_block(wl, np.arange(wl.n_int), return_triples=True)
    ml = ref["ml_max"]
    ex = _exact_bound(ref["dh"], ref["hh"], [m for _, m in wl.modes])
    assert np.all(ex >= ml * (1 - 1e-9))
    ctx = dotpe.Context(0)
    try:
        for prec in ("fp16x2", "bf16x2"):
            bank = ctx.load_bank(wl.h, wl.modes, wl.f, wl.ln_w_int, precision=prec)
            ev = ctx.set_event(bank, d=wl.d, w=wl.w, det_r=wl.det_r, det_D=wl.det_D, ext=wl.ext,
                               n_phi=wl.n_phi, ln_w_ext=wl.ln_w_ext, d_max=wl.d_max, d0=wl.d0)
            both = ev.bound().astype(np.float64)
            ev.close()
            bank.close()
            fin = np.isfinite(ex)
            top = fin & (ml >= ml.max() - 40.0)
            for name, bd, most in (("whole rows", both[0], 0.1 if prec == "fp16x2" else 1.0),
                                   ("per group", both[1], 0.05 if prec == "fp16x2" else 0.5)):
                rel = (bd - ex)[top] / ex[top]
                print(f"{cfg} SNR {snr} {prec} margin of {name}: max lnL^ML {ml.max():.3f}, exact "
                      f"bound {ex[fin].max():.3f}, bound {bd[np.isfinite(bd)].max():.3f}; within 40 "
                      f"of the max: excess median {np.median(rel):.3g}, max {np.max(rel):.3g}; "
                      f"pairs without a bound {int(np.sum(~np.isfinite(bd)))} "
                      f"({int(np.sum(~fin))} exact)", flush=True)
                assert np.all(bd >= 1.0008 * np.where(fin, ex, 0.0)), np.min(bd - 1.0008 * ex)
                assert np.all(bd >= 1.0005 * ml)
                assert np.all(~np.isfinite(bd)[~fin])
                assert np.max(rel) <= most
            # Cauchy-Schwarz over the groups and outputs: the per-group margin is the smaller
            assert np.all(both[1] <= both[0] * (1 + 1e-5) + 1e-5)
    finally:
        ctx.close()
