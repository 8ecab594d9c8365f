"""Pins of the oracle's (m, p) layout and relative-binning functions (Sec. IV
A eq. h_k with real F_kp; App. A eqs. dh_weights, hh_weights, d_h, h_h):
hat splines, exactness where the binned ratio is exactly piecewise linear,
reduction to the plain bins, equality of the (m, p) and (l, m) layouts for a
non-precessing source, and the approximation near the reference."""
import math

import numpy as np

from oracle import oracle as O
from synth import workload as W


def _full_res_products(ev, rows, R, t, phis):
    """dh, hh [rows, E, O] by direct sums over the full-resolution grid."""
    f = ev.f_full
    mm = np.array([c[1] if ev.layout == "lm" else c[0] for c in ev.chans], dtype=np.float64)
    wl = ev.wl
    if ev.layout == "lm":
        h = W.waveform_modes(f, wl.meta["mc"][rows], wl.meta["q"][rows], wl.meta["chi"][rows], wl.modes)
    else:
        raise NotImplementedError
    T = np.exp(-2j * np.pi * f[None, None, :] * t[:, :, None])
    Phi = np.exp(-1j * np.outer(phis, mm))
    dh = np.empty((len(rows), R.shape[0], len(phis)))
    hh = np.empty_like(dh)
    for a in range(len(rows)):
        hk = np.einsum("cf,ekc,oc->eokf", h[a], R, Phi) * T[:, None]
        dh[a] = np.real(np.einsum("kf,eokf->eo", ev.w_full * ev.d_full, np.conj(hk)))
        hh[a] = np.einsum("kf,eokf->eo", ev.w_full, np.abs(hk) ** 2)
    return dh, hh


def test_hat_splines():
    f = np.linspace(10.0, 100.0, 901)
    nodes = np.array([12.0, 15.0, 22.5, 40.0, 41.0, 95.0])
    s = O.hat_splines(f, nodes)
    inside = (f >= nodes[0]) & (f <= nodes[-1])
    assert np.allclose(s[:, inside].sum(0), 1.0, atol=1e-14)
    assert np.all(s[:, ~inside] == 0.0)
    idx = [int(np.argmin(np.abs(f - x))) for x in nodes]
    assert np.allclose(s[:, idx], np.eye(len(nodes)), atol=1e-12)
    # linear functions are reproduced exactly between the nodes
    g = 3.0 - 0.25 * f
    assert np.allclose((s * (3.0 - 0.25 * nodes)[:, None]).sum(0)[inside], g[inside], rtol=1e-13)


def test_rb_exact_for_piecewise_linear_ratios():
    ev = W.make_rb_event(3, 4, 2, 48, 3000, layout="lm")
    rng = np.random.default_rng(7)
    C, K = ev.h0.shape[0], ev.d_full.shape[0]
    f = ev.f_full
    al = rng.normal(size=C) + 1j * rng.normal(size=C)
    be = (rng.normal(size=C) + 1j * rng.normal(size=C)) * 1e-2
    R = rng.normal(size=(1, K, C)) + 1j * rng.normal(size=(1, K, C))
    t = ev.t0[None, :]
    mm = np.array([m for _, m in ev.chans], dtype=np.float64)
    phis = O.phase_grid(8)
    Wdh, Whh, dd = O.rb_weights(f, ev.d_full, ev.w_full, ev.h0, ev.node_idx, ev.t0)
    assert dd == np.sum(ev.w_full * np.abs(ev.d_full) ** 2)
    for lin in (True, False):
        ratio = al[:, None] + (be[:, None] * f[None, :] if lin else 0.0)
        h = ev.h0 * ratio                                              # [C, F]
        dh, hh = O.triple_inner_products_rb(h[:, ev.node_idx], R, t, f[ev.node_idx], mm, phis, Wdh, Whh)
        T = np.exp(-2j * np.pi * f[None, None, :] * t[:, :, None])
        hk = np.einsum("cf,ekc,oc->eokf", h, R, np.exp(-1j * np.outer(phis, mm))) * T[:, None]
        dh_full = np.real(np.einsum("kf,eokf->eo", ev.w_full * ev.d_full, np.conj(hk)))
        hh_full = np.einsum("kf,eokf->eo", ev.w_full, np.abs(hk) ** 2)
        # (d|h) is linear in the ratio: exact for a linear one; (h|h) is
        # quadratic: exact for a constant one
        assert np.allclose(dh, dh_full, rtol=0, atol=1e-10 * np.max(hh_full)), lin
        if not lin:
            assert np.allclose(hh, hh_full, rtol=1e-10), lin


def test_rb_reduces_to_plain_bins():
    wl = W.config_tiny(seed=2).subset(rows=np.arange(4), cols=np.arange(16))
    C, K, B = wl.h.shape[1], wl.d.shape[0], wl.d.shape[1]
    Wdh = np.broadcast_to((wl.w * wl.d)[:, None, :], (K, C, B))
    Whh = np.broadcast_to(wl.w[:, None, None, :], (K, C, C, B)).astype(np.complex128)
    R = O.response(wl.det_D, wl.modes, wl.ext)
    t = O.arrival_times(wl.det_r, wl.ext["lat"], wl.ext["lon"], wl.ext["t_geo"])
    phis = O.phase_grid(wl.n_phi)
    mm = np.array([m for _, m in wl.modes], dtype=np.float64)
    for i in range(4):
        a = O.triple_inner_products(wl.h[i], R, t, wl.f, mm, phis, wl.d, wl.w)
        b = O.triple_inner_products_rb(wl.h[i], R, t, wl.f, mm, phis, Wdh, Whh)
        assert np.allclose(a[0], b[0], rtol=1e-12, atol=1e-12 * np.max(a[1]))
        assert np.allclose(a[1], b[1], rtol=1e-12)


def test_mp_layout_equals_lm_layout():
    """A non-precessing source in the (m, p) layout (h_mp = sum_l K_{lm,p}(iota) h_lm,
    real F) gives the same inner products as the (l, m) layout with the
    inclination in the extrinsic response."""
    wl = W.config_production(seed=4, n_int=3, n_ext=24)
    rng = np.random.default_rng(1)
    ci = rng.uniform(-0.95, 0.95, 3)
    chans = W.mp_channels(wl.modes)
    phis = O.phase_grid(wl.n_phi)
    t = O.arrival_times(wl.det_r, wl.ext["lat"], wl.ext["lon"], wl.ext["t_geo"])
    m_lm = np.array([m for _, m in wl.modes], dtype=np.float64)
    m_mp = np.array([m for m, _ in chans], dtype=np.float64)
    R_mp = O.response_mp(wl.det_D, [p for _, p in chans], wl.ext)
    for i in range(3):
        Kf = O.mode_factors(wl.modes, np.array([ci[i]]))[0]                 # [C, 2]
        h_mp = np.zeros((len(chans), len(wl.f)), dtype=np.complex128)
        for c, (l, m) in enumerate(wl.modes):
            for p in (0, 1):
                h_mp[chans.index((m, p))] += Kf[c, p] * wl.h[i, c]
        ext = dict(wl.ext, cos_iota=np.full(wl.n_ext, ci[i]))
        R_lm = O.response(wl.det_D, wl.modes, ext)
        a = O.triple_inner_products(wl.h[i], R_lm, t, wl.f, m_lm, phis, wl.d, wl.w)
        b = O.triple_inner_products(h_mp, R_mp, t, wl.f, m_mp, phis, wl.d, wl.w)
        assert np.allclose(a[0], b[0], rtol=1e-10, atol=1e-10 * np.max(a[1]))
        assert np.allclose(a[1], b[1], rtol=1e-10)


def test_synth_mp_bank_matches_oracle_factors():
    """The input generator's (m, p) bank (its own -2Y_lm) against the oracle's factors."""
    f = W.freq_bins(32, 20.0, 200.0)
    mc, q, chi = np.array([5.0, 8.0]), np.array([0.5, 0.8]), np.array([0.1, -0.3])
    ci = np.array([0.3, -0.7])
    h_mp, chans = W.waveform_mp(f, mc, q, chi, ci, W.MODES_HM)
    h_lm = W.waveform_modes(f, mc, q, chi, W.MODES_HM)
    for i in range(2):
        Kf = O.mode_factors(W.MODES_HM, ci[i:i + 1])[0]
        ref = np.zeros_like(h_mp[i])
        for c, (l, m) in enumerate(W.MODES_HM):
            for p in (0, 1):
                ref[chans.index((m, p))] += Kf[c, p] * h_lm[i, c]
        assert np.allclose(h_mp[i], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_rb_close_to_full_resolution_near_the_reference():
    """Bank rows within 1% of the reference chirp mass and extrinsic samples
    within 0.5 ms of its arrival time: relative binning on 64 nodes against
    direct sums over 6000 frequencies (the paper quotes ~1% accuracy at ~100
    bins)."""
    ev = W.make_rb_event(5, 6, 12, 64, 6000, layout="lm", snr=20.0)
    wl = ev.wl
    Wdh, Whh, _ = O.rb_weights(ev.f_full, ev.d_full, ev.w_full, ev.h0, ev.node_idx, ev.t0)
    R = O.response(wl.det_D, wl.modes, wl.ext)
    t = O.arrival_times(wl.det_r, wl.ext["lat"], wl.ext["lon"], wl.ext["t_geo"])
    phis = O.phase_grid(wl.n_phi)
    mm = np.array([m for _, m in wl.modes], dtype=np.float64)
    rows = np.arange(6)
    dh_f, hh_f = _full_res_products(ev, rows, R, t, phis)
    for a in rows:
        dh, hh = O.triple_inner_products_rb(wl.h[a], R, t, wl.f, mm, phis, Wdh, Whh)
        scale = np.max(hh_f[a])
        # (measured: a few 1e-6 and up to 3e-5 of (h|h))
        assert np.max(np.abs(dh - dh_f[a])) <= 1e-3 * scale
        assert np.max(np.abs(hh - hh_f[a])) <= 1e-3 * scale
