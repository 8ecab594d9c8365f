"""dotpe_evidence_static (the entry point that allocates no device memory)
against dotpe_set_event + dotpe_evidence on the same events, through the C
ABI: two calls in a row, the second with a smaller event on another bank,
so that whatever the first call left in the shared scratch must not leak
into the second."""
import numpy as np
import pytest

from synth import workload as W

pytestmark = pytest.mark.gpu

FLOAT_KEYS = ("ln_z", "ln_z_upper", "max_lnl_ml", "ln_sum_p", "ln_sum_p2", "dd", "max_ln_p",
              "cut_delta_used")
INT_KEYS = ("n_pairs", "n_pairs_bounded", "n_triples_marg", "precision", "topk_count",
            "topk_exact", "n_passes")


def _kw(wl, **extra):
    return dict(d=wl.d, w=wl.w, det_r=wl.det_r, det_D=wl.det_D, ext=wl.ext, n_phi=wl.n_phi,
                ln_w_ext=wl.ln_w_ext, d_max=wl.d_max, d0=wl.d0, **extra)


def test_static_evidence_matches_allocating_path():
    from paper_2507_16022_amd import dotpe
    ctx = dotpe.Context(0)
    big = W.config_production(seed=40, n_int=2048, n_ext=1024, snr=25.0, random_weights=True)
    small = W.config_tiny(seed=41, n_int=96, n_ext=130, random_weights=True)
    cases = [(big, "fp16x2", dict(cut_delta=30.0, top_k=32, topk_window=20.0)),
             (small, "fp64", dict(top_k=8))]
    for wl, prec, extra in cases:
        bank = ctx.load_bank(wl.h, wl.modes, wl.f, wl.ln_w_int, precision=prec)
        held = ctx.device_bytes()
        got = ctx.evidence_static(bank, **_kw(wl, **extra))
        assert ctx.device_bytes() == held          # nothing allocated through the context
        ev = ctx.set_event(bank, **_kw(wl, **extra))
        ref = ev.evidence()
        ev.close()
        print(f"static {prec} {wl.n_int}x{wl.n_ext}: ln Z {got['ln_z']:.12f} vs {ref['ln_z']:.12f}, "
              f"top-k {got['topk_count']}", flush=True)
        assert got["n_pairs"] == wl.n_int * wl.n_ext
        for k in INT_KEYS:
            assert got[k] == ref[k], k
        for k in FLOAT_KEYS:
            assert abs(got[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), k
        assert got["topk_count"] > 0
        assert np.array_equal(got["topk_i"], ref["topk_i"])
        assert np.array_equal(got["topk_e"], ref["topk_e"])
        assert np.array_equal(got["topk_o"], ref["topk_o"])
        assert np.max(np.abs(got["topk_lnp"] - ref["topk_lnp"])) <= 1e-12 * max(1.0, abs(ref["ln_z"]))
        bank.close()
    # an event larger than the scratch is refused before anything runs
    huge = W.config_production(seed=42, n_int=65536, n_ext=4096, with_bank=False)
    bank = ctx.load_bank(np.zeros((65536, 5, 256), dtype=np.complex128), W.MODES_HM, huge.f,
                         precision="fp16x2")
    with pytest.raises(dotpe.DotpeError) as e:
        ctx.evidence_static(bank, **_kw(huge))
    assert e.value.code == dotpe.E_TOO_LARGE
    bank.close()
    ctx.close()
