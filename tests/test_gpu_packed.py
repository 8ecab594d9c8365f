"""Packed serving batches on the GPU.

A server with one slot and batches of up to 8 events runs events of every
kind together -- large ones that take the bound pass and the survivor pass,
small ones that take the fused kernel's fast pass, a quiet one whose largest
lnL^ML stays below the cut (every tile takes the coefficient route), one with
the cut off, one with a scattered bank subset, two-detector and
three-detector networks -- so that each stage of the evidence pass is one
launch over the tiles of several events.  Each result must equal the same
event evaluated alone with dotpe_evidence: the events keep their own grids
and decisions and every sum is taken in a fixed order.
"""
import numpy as np
import pytest

from synth import workload as W

pytestmark = pytest.mark.gpu

TOL = 1e-9
N_BANK = 8192


@pytest.fixture(scope="module")
def setup():
    from paper_2507_16022_amd import dotpe
    ctx = dotpe.Context(0)
    bank_wl = W.make_workload(13, n_int=N_BANK, n_ext=8, n_bins=256, modes=W.MODES_HM,
                              dets="HLV", n_phi=32, snr=20.0, mc_range=(5.0, 80.0),
                              q_range=(0.1, 1.0), chi_range=(-0.9, 0.9))
    bank = ctx.load_bank(bank_wl.h, bank_wl.modes, bank_wl.f, precision="fp16x2")
    yield dotpe, ctx, bank, bank_wl
    bank.close()
    ctx.close()


def event(bank_wl, seed, n_ext, dets, snr, cut=30.0, top_k=64, **sub):
    ev = W.make_workload(seed, n_int=8, n_ext=n_ext, n_bins=256, modes=W.MODES_HM, dets=dets,
                         n_phi=32, snr=snr, mc_range=(5.0, 80.0), q_range=(0.1, 1.0),
                         chi_range=(-0.9, 0.9), with_bank=False)
    assert np.allclose(ev.f, bank_wl.f)
    return dict(d=ev.d, w=ev.w, det_r=ev.det_r, det_D=ev.det_D, ext=ev.ext, n_phi=ev.n_phi,
                ln_w_ext=ev.ln_w_ext, d_max=ev.d_max, d0=ev.d0, cut_delta=cut, top_k=top_k,
                topk_window=20.0, **sub)


def alone(ctx, bank, kw):
    ev = ctx.set_event(bank, **kw)
    r = ev.evidence()
    ev.close()
    return r


def test_packed_batch_matches_alone(setup):
    dotpe, ctx, bank, bank_wl = setup
    rng = np.random.default_rng(17)
    scattered = np.sort(rng.choice(N_BANK, 3000, replace=False)).astype(np.int64)
    specs = [
        # the slot is idle when this one arrives: it runs alone while the
        # others queue, and they then share batches
        event(bank_wl, 500, 2048, "HLV", 18.0, sub_start=0, sub_count=4096),
        event(bank_wl, 501, 4096, "HLV", 20.0, sub_start=0, sub_count=N_BANK),    # bound pass
        event(bank_wl, 502, 4096, "HL", 12.0, sub_start=0, sub_count=N_BANK),     # bound pass
        event(bank_wl, 503, 512, "HLV", 15.0, sub_start=100, sub_count=1024),     # fast pass
        event(bank_wl, 504, 1024, "HLV", 4.0, sub_start=2000, sub_count=2048),    # quiet
        event(bank_wl, 505, 256, "HL", 25.0, cut=0.0, sub_start=7000, sub_count=512),
        event(bank_wl, 506, 96, "HLV", 22.0, sub_idx=scattered),
        event(bank_wl, 507, 1000, "HL", 9.0, sub_start=33, sub_count=777),
        event(bank_wl, 508, 2048, "HLV", 30.0, sub_start=4096, sub_count=4096),
    ]
    # no work budget: the large events share batches too
    srv = dotpe.Server(ctx, bank, n_slots=1, pool_bytes=8 << 30, max_batch=8, batch_pairs=1 << 40)
    tickets = [srv.submit(**kw) for kw in specs]
    got = [srv.wait(t) for t in tickets]
    srv.close()
    batches = [info["batch"] for _, info in got]
    print(f"batch sizes {batches}", flush=True)
    assert max(batches) >= 3, batches
    worst = 0.0
    for q, ((r, info), kw) in enumerate(zip(got, specs)):
        ref = alone(ctx, bank, kw)
        assert info["status"] == 0 and info["slot"] == 0
        d = abs(r["ln_z"] - ref["ln_z"])
        worst = max(worst, d, abs(r["ln_z_upper"] - ref["ln_z_upper"]))
        print(f"event {q}: ln Z {r['ln_z']:.9f} alone {ref['ln_z']:.9f}, passes "
              f"{r['n_passes']}, tiles rerun {r['n_tiles_rerun']}, listed {r['n_tiles_listed']}, "
              f"bounded {r['n_pairs_bounded']}/{r['n_pairs']}", flush=True)
        assert d <= TOL
        assert abs(r["ln_z_upper"] - ref["ln_z_upper"]) <= TOL
        for k in ("ln_sum_p2", "ln_sum_p2_triples", "ln_sum_row2", "ln_sum_col2", "max_lnl_ml"):
            assert abs(r[k] - ref[k]) <= TOL, k
        for k in ("n_pairs", "n_pairs_bounded", "n_triples_marg", "n_tiles_rerun",
                  "n_tiles_listed", "n_passes", "topk_count", "topk_exact"):
            assert r[k] == ref[k], k
        n = r["topk_count"]
        lnp = r["topk_lnp"][:n]
        assert np.all(np.diff(lnp) <= 0) and np.all(lnp >= r["max_ln_p"] - 20.0)
        if r["topk_exact"]:
            assert np.array_equal(r["topk_i"][:n], ref["topk_i"][:n])
            assert np.array_equal(r["topk_e"][:n], ref["topk_e"][:n])
            assert np.allclose(lnp, ref["topk_lnp"][:n], atol=TOL, rtol=0)
        # else the candidate buffer overflowed (a quiet event, where most
        # pairs lie within the window of the largest): which candidates it
        # kept depends on timing, alone as well as packed, and the result
        # says so
    print(f"largest |d ln Z| packed vs alone: {worst:.3e}", flush=True)
    # the kinds of pass the batch was meant to mix did occur
    kinds = [alone_kind(r) for r, _ in got]
    assert {"bound", "fast", "nocut"} <= set(kinds), kinds


def alone_kind(r):
    if r["cut_delta_used"] <= 0.0:
        return "nocut"
    return "bound" if r["n_tiles_listed"] > 0 else "fast"


@pytest.mark.parametrize("precision", ["fp64", "bf16x2"])
def test_packed_batch_other_precisions(precision):
    """The packed launches of the FP64 and BF16x2 kernels (pilot, fast pass,
    coefficient route): small events served in one batch equal each event
    alone."""
    from paper_2507_16022_amd import dotpe
    ctx = dotpe.Context(0)
    bank_wl = W.make_workload(21, n_int=2048, n_ext=8, n_bins=256, modes=W.MODES_HM, dets="HLV",
                              n_phi=32, snr=20.0, mc_range=(5.0, 80.0), q_range=(0.1, 1.0),
                              chi_range=(-0.9, 0.9))
    bank = ctx.load_bank(bank_wl.h, bank_wl.modes, bank_wl.f, precision=precision)
    specs = [
        event(bank_wl, 600, 512, "HLV", 18.0, sub_start=0, sub_count=2048),
        event(bank_wl, 601, 256, "HL", 12.0, sub_start=100, sub_count=700),
        event(bank_wl, 602, 384, "HLV", 5.0, sub_start=1024, sub_count=1024),
        event(bank_wl, 603, 200, "HLV", 25.0, cut=0.0, sub_start=7, sub_count=300),
        event(bank_wl, 604, 96, "HL", 22.0, sub_start=1500, sub_count=548),
    ]
    srv = dotpe.Server(ctx, bank, n_slots=1, pool_bytes=4 << 30, max_batch=8, batch_pairs=1 << 40)
    tickets = [srv.submit(**kw) for kw in specs]
    got = [srv.wait(t) for t in tickets]
    srv.close()
    batches = [info["batch"] for _, info in got]
    print(f"{precision}: batch sizes {batches}", flush=True)
    assert max(batches) >= 2, batches
    for (r, info), kw in zip(got, specs):
        ref = alone(ctx, bank, kw)
        assert info["status"] == 0
        assert abs(r["ln_z"] - ref["ln_z"]) <= TOL and abs(r["ln_z_upper"] - ref["ln_z_upper"]) <= TOL
        for k in ("n_pairs", "n_pairs_bounded", "n_triples_marg", "n_passes", "topk_count"):
            assert r[k] == ref[k], k
        if r["topk_exact"]:
            n = r["topk_count"]
            assert np.array_equal(r["topk_i"][:n], ref["topk_i"][:n])
            assert np.array_equal(r["topk_e"][:n], ref["topk_e"][:n])
    bank.close()
    ctx.close()


def test_packed_batch_with_a_failing_event(setup):
    """An event whose staging fails on the device (strain so large that the
    extrinsic operand overflows, which the conversion kernel flags) reports
    its error; the events batched with it complete as they would alone."""
    dotpe, ctx, bank, bank_wl = setup
    good = [event(bank_wl, 700 + q, 256, "HLV", 15.0, sub_start=512 * q, sub_count=512)
            for q in range(3)]
    bad = event(bank_wl, 710, 256, "HLV", 15.0, sub_start=0, sub_count=512)
    bad["d"] = bad["d"].copy()
    bad["d"][0, 5] = 1e308
    srv = dotpe.Server(ctx, bank, n_slots=1, pool_bytes=4 << 30, max_batch=8, batch_pairs=1 << 40)
    specs = [good[0], bad, good[1], good[2]]
    tickets = [srv.submit(**kw) for kw in specs]
    outcomes = []
    for t in tickets:
        try:
            outcomes.append(srv.wait(t))
        except dotpe.DotpeError as e:
            outcomes.append(e)
    srv.close()
    assert isinstance(outcomes[1], dotpe.DotpeError) and outcomes[1].code == dotpe.E_NUMERIC
    for q, kw in ((0, good[0]), (2, good[1]), (3, good[2])):
        r, info = outcomes[q]
        ref = alone(ctx, bank, kw)
        assert info["status"] == 0
        assert abs(r["ln_z"] - ref["ln_z"]) <= TOL
