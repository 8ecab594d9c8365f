"""The fused evidence pass at the large shape (2^20 bank waveforms x 16384
extrinsic samples, 3 detectors, 5 modes, 256 bins, 32 phases, SNR 20),
in the launch configuration the benchmark times, checked against
independent results:

* the plain FP64 GPU path on the same event (FP64 operands and MFMA): ln Z
  within 1e-3, each ln Z inside the other's certified interval;
* the oracle, pair by pair, on the 64 best pairs the fused pass returns and
  on 512 pairs drawn at random, half of them in bank rows whose operand
  offsets pass 2^31 elements;
* the same event over a scattered subset (every bank row, in a random
  order): ln Z and the top pairs do not depend on the row order (eq. Z_sum
  is a sum over pairs).
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import workload as W

pytestmark = pytest.mark.gpu

N_INT, N_EXT, SEED, SNR = 1 << 20, 16384, 3, 20.0
CUT, WINDOW, TOPK = 40.0, 20.0, 64
TOL = 1e-3


@pytest.fixture(scope="module")
def large():
    import torch
    from paper_2507_16022_amd import dotpe
    wl = W.config_large(seed=SEED, snr=SNR, with_bank=False)
    h = W.bank_on_device(torch, wl.meta["mc"], wl.meta["q"], wl.meta["chi"], wl.f, wl.modes)
    ctx = dotpe.Context(0)
    banks = {p: ctx.load_bank(h, wl.modes, wl.f, precision=p) for p in ("fp16x2", "fp64")}
    yield wl, h, ctx, banks
    for b in banks.values():
        b.close()
    ctx.close()


def _event(ctx, bank, wl, **kw):
    return ctx.set_event(bank, d=wl.d, w=wl.w, det_r=wl.det_r, det_D=wl.det_D, ext=wl.ext,
                         n_phi=wl.n_phi, ln_w_ext=wl.ln_w_ext, d_max=wl.d_max, d0=wl.d0, **kw)


def _oracle_pairs(wl, h, pairs):
    """ln Lbar of (bank row, extrinsic sample) pairs by the oracle, with the
    bank rows copied from the generated device bank."""
    rows = np.unique(pairs[:, 0])
    hr = h[rows].cpu().numpy()
    sub = W.Workload(wl.modes, wl.f, hr[..., 0] + 1j * hr[..., 1], np.zeros(len(rows)), wl.det_r,
                     wl.det_D, wl.d, wl.w, wl.ext, wl.ln_w_ext, wl.n_phi, wl.d_max, wl.d0)
    where = {r: a for a, r in enumerate(rows)}
    out = np.empty(len(pairs))
    for q, (i, e) in enumerate(pairs):
        out[q] = O.eval_pairs_block(sub, [where[i]], ext_idx=[e])["lnl"][0, 0]
    return out


def test_large_evidence_vs_fp64_and_oracle(large):
    wl, h, ctx, banks = large
    res = {}
    for p, b in banks.items():
        ev = _event(ctx, b, wl, cut_delta=CUT, top_k=TOPK, topk_window=WINDOW)
        res[p] = ev.evidence()
        ev.close()
        r = res[p]
        print(f"large {p}: ln Z {r['ln_z']:.9f} upper {r['ln_z_upper']:.9f} bounded "
              f"{r['n_pairs_bounded']}/{r['n_pairs']} fused {r['t_fused_ms']:.1f} ms "
              f"passes {r['n_passes']}", flush=True)
        assert r["n_pairs"] == N_INT * N_EXT
        assert r["ln_z_upper"] - r["ln_z"] <= 1e-4
        assert r["topk_count"] == TOPK and r["topk_exact"] == 1
    a, b = res["fp16x2"], res["fp64"]
    assert abs(a["ln_z"] - b["ln_z"]) <= TOL
    assert a["ln_z"] <= b["ln_z_upper"] + TOL and b["ln_z"] <= a["ln_z_upper"] + TOL
    assert abs(a["max_lnl_ml"] - b["max_lnl_ml"]) <= TOL
    # every pair within TOL of the FP64 value keeps the sorted values within TOL
    assert np.max(np.abs(a["topk_lnp"] - b["topk_lnp"])) <= TOL
    # the returned best pairs, one by one against the oracle (ln w = 0 here)
    pairs = np.stack([a["topk_i"], a["topk_e"]], -1)
    ref = _oracle_pairs(wl, h, pairs)
    err = np.abs(a["topk_lnp"] - ref)
    print(f"large fp16x2 top-{TOPK} vs oracle: max |d ln p| = {err.max():.3e}", flush=True)
    assert err.max() <= TOL


def test_large_random_pairs_vs_oracle(large):
    """512 pairs through the materialising pass on the resident banks, half
    of them in rows whose split-operand offset i * K2 passes 2^31."""
    wl, h, ctx, banks = large
    rng = np.random.default_rng(7)
    k2 = 2 * len(wl.modes) * 256
    lo = (1 << 31) // k2 + 1
    rows = np.concatenate([rng.choice(lo, 8, replace=False), rng.choice(np.arange(lo, N_INT), 8,
                                                                      replace=False)])
    cols = np.sort(rng.choice(N_EXT, 32, replace=False))
    sub_ext = {k: v[cols] for k, v in wl.ext.items()}
    got = {}
    for p, b in banks.items():
        ev = ctx.set_event(b, d=wl.d, w=wl.w, det_r=wl.det_r, det_D=wl.det_D, ext=sub_ext,
                           n_phi=wl.n_phi, ln_w_ext=wl.ln_w_ext[cols], d_max=wl.d_max, d0=wl.d0,
                           sub_idx=rows)
        got[p] = ev.eval_lnl()["lnl"]
        ev.close()
    pairs = np.array([(i, e) for i in rows for e in cols])
    ref = _oracle_pairs(wl, h, pairs).reshape(len(rows), len(cols))
    e16 = np.abs(got["fp16x2"] - ref)
    e64 = np.abs(got["fp64"] - ref)
    print(f"large random pairs: max |d lnLbar| fp16x2 {e16.max():.3e} (rows past 2^31 elements "
          f"{e16[8:].max():.3e}), fp64 {e64.max():.3e}", flush=True)
    assert e16.max() <= TOL
    assert e64.max() <= 1e-6


def test_large_scattered_rows_same_evidence(large):
    """Every bank row in a random order (an explicit index list): ln Z and the
    best pairs equal those of the contiguous range."""
    wl, h, ctx, banks = large
    b = banks["fp16x2"]
    ev = _event(ctx, b, wl, cut_delta=CUT, top_k=TOPK, topk_window=WINDOW)
    r0 = ev.evidence()
    ev.close()
    perm = np.random.default_rng(11).permutation(N_INT).astype(np.int64)
    ev = _event(ctx, b, wl, cut_delta=CUT, top_k=TOPK, topk_window=WINDOW, sub_idx=perm)
    r1 = ev.evidence()
    ev.close()
    print(f"large scattered rows: ln Z {r1['ln_z']:.12f} vs {r0['ln_z']:.12f}, fused "
          f"{r1['t_fused_ms']:.1f} ms vs {r0['t_fused_ms']:.1f} ms", flush=True)
    assert abs(r1["ln_z"] - r0["ln_z"]) <= 1e-8
    assert abs(r1["ln_sum_p2"] - r0["ln_sum_p2"]) <= 1e-8
    assert r1["topk_count"] == r0["topk_count"]
    assert np.array_equal(r1["topk_i"], r0["topk_i"]) and np.array_equal(r1["topk_e"], r0["topk_e"])
    assert np.max(np.abs(r1["topk_lnp"] - r0["topk_lnp"])) <= 1e-9
