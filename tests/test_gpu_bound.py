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
    # the same pairs are bounded (the same bound from the same accumulators);
    # the survivors' inner products are summed in FP64 on one route and in
    # FP32 on the matrix cores on the other, so the rest agrees to rounding
    assert a["n_pairs_bounded"] == b["n_pairs_bounded"]
    assert abs(a["n_triples_marg"] - b["n_triples_marg"]) <= 1e-3 * b["n_triples_marg"] + 2
    for k in ("ln_z", "ln_z_upper", "ln_sum_p2", "max_lnl_ml", "max_ln_p", "ln_sum_p2_triples",
              "ln_sum_row2", "ln_sum_col2"):
        assert abs(a[k] - b[k]) <= 1e-3, k
    assert a["topk_count"] == b["topk_count"] and a["topk_count"] > 0
    assert np.max(np.abs(a["topk_lnp"] - b["topk_lnp"])) <= 1e-3
    # (with a cut narrower than the top-k window, cut pairs may lie in the window)
    assert a["topk_exact"] == b["topk_exact"] == (1 if cut >= 30.0 else b["topk_exact"])
    assert a["ln_z_upper"] - a["ln_z"] <= 1e-4
    if prec == "fp16x2":
        c = _run(ctx, banks["fp64"], wl, **kw)
        print(f"   fp64 path: ln Z {c['ln_z']:.10f}; top-16 |d ln p| bound route "
              f"{np.max(np.abs(a['topk_lnp'][:16] - c['topk_lnp'][:16])):.2e}, fused route "
              f"{np.max(np.abs(b['topk_lnp'][:16] - c['topk_lnp'][:16])):.2e}", flush=True)
        for r in (a, b):
            assert abs(r["ln_z"] - c["ln_z"]) <= 1e-3
            assert np.max(np.abs(r["topk_lnp"][:16] - c["topk_lnp"][:16])) <= 1e-3
