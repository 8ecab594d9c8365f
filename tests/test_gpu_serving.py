"""Serving calls (dotpe_submit / dotpe_poll / dotpe_wait) on the GPU.

Events of different sizes, detector counts and bank subsets are submitted
together to a server whose pool holds only a few of them at once, so that
admission queues; each result must equal the same event evaluated alone
with dotpe_evidence (the cut is certified, so only which pairs get bounded
may differ, which moves ln Z by far less than the tolerance below).
"""
import numpy as np
import pytest

from synth import workload as W

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def setup():
    from paper_2507_16022_amd import dotpe
    ctx = dotpe.Context(0)
    bank_wl = W.make_workload(11, n_int=3072, n_ext=8, n_bins=256, modes=W.MODES_HM, dets="HLV",
                              n_phi=32, snr=20.0, mc_range=(5.0, 80.0), q_range=(0.1, 1.0),
                              chi_range=(-0.9, 0.9))
    bank = ctx.load_bank(bank_wl.h, bank_wl.modes, bank_wl.f, precision="fp16x2")
    yield dotpe, ctx, bank, bank_wl
    bank.close()
    ctx.close()


def event_kwargs(bank_wl, seed, n_ext, dets, snr, sub_start, sub_count, cut=30.0, top_k=64):
    ev = W.make_workload(seed, n_int=8, n_ext=n_ext, n_bins=256, modes=W.MODES_HM, dets=dets,
                         n_phi=32, snr=snr, mc_range=(5.0, 80.0), q_range=(0.1, 1.0),
                         chi_range=(-0.9, 0.9), with_bank=False)
    assert np.allclose(ev.f, bank_wl.f)
    return dict(d=ev.d, w=ev.w, det_r=ev.det_r, det_D=ev.det_D, ext=ev.ext, n_phi=ev.n_phi,
                ln_w_ext=ev.ln_w_ext, d_max=ev.d_max, d0=ev.d0, sub_start=sub_start,
                sub_count=sub_count, cut_delta=cut, top_k=top_k, topk_window=20.0)


def alone(ctx, bank, kw):
    ev = ctx.set_event(bank, **kw)
    r = ev.evidence()
    ev.close()
    return r


def same(a, b):
    assert abs(a["ln_z"] - b["ln_z"]) <= TOL
    for k in ("ln_sum_p2_triples", "ln_sum_row2", "ln_sum_col2"):
        assert abs(a[k] - b[k]) <= TOL, k
    assert a["max_lnl_ml"] == pytest.approx(b["max_lnl_ml"], abs=TOL)
    assert a["n_pairs"] == b["n_pairs"]
    assert a["topk_count"] == b["topk_count"]
    n = a["topk_count"]
    assert np.array_equal(a["topk_i"][:n], b["topk_i"][:n])
    assert np.array_equal(a["topk_e"][:n], b["topk_e"][:n])
    assert np.allclose(a["topk_lnp"][:n], b["topk_lnp"][:n], atol=TOL, rtol=0)


def test_results_same_alone_and_in_the_mix(setup):
    dotpe, ctx, bank, bank_wl = setup
    rng = np.random.default_rng(5)
    specs = []
    for q in range(10):
        n_ext = int(rng.choice([96, 512, 1024, 2048]))
        dets = "HLV" if q % 2 else "HL"
        count = int(rng.integers(64, 3072))
        start = int(rng.integers(0, 3072 - count + 1))
        specs.append(event_kwargs(bank_wl, 100 + q, n_ext, dets, float(rng.uniform(8, 30)),
                                  start, count))
    srv_probe = dotpe.Server(ctx, bank, n_slots=1, pool_bytes=1 << 30)
    sizes = [srv_probe.event_bytes(**kw) for kw in specs]
    srv_probe.close()
    # a pool for about two of the largest events: admission has to queue
    pool = 2 * max(sizes) + (1 << 20)
    srv = dotpe.Server(ctx, bank, n_slots=4, pool_bytes=pool)
    tickets = [srv.submit(**kw) for kw in specs]
    got = [srv.wait(t) for t in tickets]
    srv.close()
    ref = [alone(ctx, bank, kw) for kw in specs]
    starts = []
    for (r, info), rr, nb in zip(got, ref, sizes):
        same(r, rr)
        assert info["status"] == 0 and 0 <= info["slot"] < 4 and info["bytes"] == nb
        assert info["t_submit_ms"] <= info["t_start_ms"] <= info["t_done_ms"]
        starts.append(info["t_start_ms"])
    # first in, first out
    assert starts == sorted(starts)


def test_poll_and_rejections(setup):
    dotpe, ctx, bank, bank_wl = setup
    kw = event_kwargs(bank_wl, 300, 256, "HLV", 15.0, 0, 1024)
    srv = dotpe.Server(ctx, bank, n_slots=2, pool_bytes=1 << 30)
    need = srv.event_bytes(**kw)
    t = srv.submit(**kw)
    r, info = srv.wait(t)
    same(r, alone(ctx, bank, kw))
    with pytest.raises(dotpe.DotpeError) as e:     # collected tickets are forgotten
        srv.poll(t)
    assert e.value.code == dotpe.E_INVALID_ARG
    with pytest.raises(dotpe.DotpeError) as e:     # invalid events are refused at submit
        srv.submit(**dict(kw, n_phi=0))
    assert e.value.code == dotpe.E_INVALID_ARG
    srv.close()
    small = dotpe.Server(ctx, bank, n_slots=1, pool_bytes=need // 2)
    with pytest.raises(dotpe.DotpeError) as e:     # larger than the whole pool
        small.submit(**kw)
    assert e.value.code == dotpe.E_ADMISSION
    # an event submitted and never waited for is run and dropped at close
    small2 = dotpe.Server(ctx, bank, n_slots=1, pool_bytes=need + (1 << 20))
    small2.submit(**kw)
    small2.close()


def test_served_event_vs_oracle(setup):
    """One event through the server, next to another it overlaps with,
    against the oracle (eq. Z_sum over eq. lnl_dist_marginalized): ln Z, the
    largest lnL^ML, and the returned top pairs' ln p, each checked at its
    (i, e) and as the set of the largest values."""
    from oracle import oracle as O
    dotpe, ctx, bank, bank_wl = setup
    start, count, n_ext, k = 1200, 40, 64, 8
    kw = event_kwargs(bank_wl, 321, n_ext, "HLV", 15.0, start, count, cut=0.0, top_k=k)
    other = event_kwargs(bank_wl, 322, 512, "HL", 20.0, 0, 3072)
    srv = dotpe.Server(ctx, bank, n_slots=2, pool_bytes=1 << 30)
    t_other = srv.submit(**other)
    t = srv.submit(**kw)
    r, _ = srv.wait(t)
    srv.wait(t_other)
    srv.close()
    wl = W.Workload(bank_wl.modes, bank_wl.f, bank_wl.h[start:start + count], np.zeros(count),
                    kw["det_r"], kw["det_D"], kw["d"], kw["w"], kw["ext"], kw["ln_w_ext"],
                    kw["n_phi"], kw["d_max"], kw["d0"])
    ref = O.evidence(wl, k=k)
    print(f"served event: ln Z {r['ln_z']:.8f} vs oracle {ref['ln_z']:.8f}", flush=True)
    assert abs(r["ln_z"] - ref["ln_z"]) <= 1e-3
    assert abs(r["max_lnl_ml"] - ref["max_lnl_ml"]) <= 1e-3
    n = r["topk_count"]
    assert n == k
    i = r["topk_i"][:n] - start
    e = r["topk_e"][:n]
    assert np.all((i >= 0) & (i < count))
    assert np.max(np.abs(r["topk_lnp"][:n] - ref["lnp"][i, e])) <= 1e-3
    assert np.max(np.abs(r["topk_lnp"][:n] - ref["topk_lnp"])) <= 1e-3
