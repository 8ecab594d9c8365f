"""Pins of the FP64 oracle against facts fixed by the paper and mathematics.

Each test names the passage (section / equation) it pins.  None of them
re-types the oracle's own formula: they use closed forms, invariants,
identities, an independent forward simulator or brute-force loops.
"""
import cmath
import math

import numpy as np
import pytest
from scipy import special

from oracle import oracle as O
from synth import workload as W


@pytest.fixture(scope="module")
def tiny():
    return W.config_tiny(seed=0)


# ---------------------------------------------------------------- P1 ------
@pytest.mark.parametrize("modes,dets,snr", [(W.MODES_22, "HL", 15.0), (W.MODES_HM, "HLV", 20.0),
                                            (W.MODES_HM, "HLV", 50.0)])
def test_zero_noise_injection_rho2_over_2(modes, dets, snr):
    """eq. (lnlike_ieo_arb_dL), (bestfit_lnl): for noise-free data equal to
    the template at the true (i, e, o, D), lnL(D_true) = lnL^ML = rho^2/2."""
    wl = W.make_workload(11, n_int=4, n_ext=4, n_bins=128, modes=modes, dets=dets, n_phi=16,
                         snr=snr, mc_range=(8.0, 30.0), q_range=(0.2, 1.0),
                         chi_range=(-0.5, 0.5), noise_on=False, in_bank=True)
    m = wl.meta
    r = O.eval_pairs_block(wl, [0], ext_idx=[0], return_triples=True)
    dh = r["dh"][0, 0, m["inj_o"]]
    hh = r["hh"][0, 0, m["inj_o"]]
    assert O.lnl_at_distance(dh, hh, m["inj_dist"], wl.d0) == pytest.approx(snr ** 2 / 2, rel=1e-12)
    assert float(O.lnl_ml(dh, hh)) == pytest.approx(snr ** 2 / 2, rel=1e-12)
    # and the injection attains the maximum over the phase grid for that pair
    # (22-only is symmetric under phi -> phi + pi, so compare values)
    ml = O.lnl_ml(r["dh"][0, 0], r["hh"][0, 0])
    assert ml[m["inj_o"]] == pytest.approx(np.max(ml), rel=1e-12)


# ---------------------------------------------------------------- P2 ------
def test_cauchy_schwarz(tiny):
    """(d|h)^2 <= (d|d)(h|h) for every triple (inner product of Sec. III A)."""
    wl = tiny.subset(rows=np.arange(8), cols=np.arange(32))
    r = O.eval_pairs_block(wl, np.arange(8), return_triples=True)
    dd = O.data_inner(wl.d, wl.w)
    assert np.all(r["dh"] ** 2 <= dd * r["hh"] * (1 + 1e-12))
    # lnL^ML is therefore bounded by (d|d)/2
    assert np.all(r["ml_max"] <= 0.5 * dd * (1 + 1e-12))


# ---------------------------------------------------------------- P3 ------
def test_zero_data_closed_form():
    """d = 0: Lbar = 3 int_0^1 r^2 exp(-x0^2/r^2) dr
    = exp(-x0^2)(1 - 2 x0^2) + 2 sqrt(pi) x0^3 erfc(x0), x0 = (d0/Dmax) sqrt(hh/2)
    (eq. lnl_dist_marginalized with a D^2 prior)."""
    dmax = 5000.0
    hh = np.array([1e2, 1e5, 1e6, 1e7, 3e7, 1e8, 4e8])
    x0 = np.sqrt(hh / 2) / dmax
    exact = np.exp(-x0 ** 2) * (1 - 2 * x0 ** 2) + 2 * math.sqrt(math.pi) * x0 ** 3 * special.erfc(x0)
    got = O.ln_dist_marg(np.zeros_like(hh), hh, dmax, 1.0, n_nodes=2000)
    assert np.allclose(got, np.log(exact), atol=1e-11, rtol=0)


# ---------------------------------------------------------------- P4 ------
def test_phase_grid_bessel_identity():
    """22-only: dh_o = |X| cos(2 phi_o + a), hh_o constant, and the grid
    average of exp(A cos(2 phi + a)) equals
    I_0(A) + 2 sum_k I_{kN/2}(A) cos(k N a / 2)  (Fourier series of e^{A cos t})."""
    wl = W.config_tiny(seed=3, n_int=6, n_ext=6, snr=12.0)
    r = O.eval_pairs_block(wl, np.arange(6), return_triples=True)
    N = wl.n_phi
    phis = 2 * np.pi * np.arange(N) / N
    D, q = O.distance_nodes(wl.d_max)
    u = wl.d0 / D
    for i in range(6):
        for e in range(6):
            dh, hh = r["dh"][i, e], r["hh"][i, e]
            assert np.allclose(hh, hh[0], rtol=1e-12)
            c = np.sum(dh * np.exp(-2j * phis)) * 2 / N      # dh = Re(c e^{2i phi})
            amp, a = abs(c), cmath.phase(c)
            assert np.allclose(dh, amp * np.cos(2 * phis + a), atol=1e-9 * max(1.0, amp))
            A = u * amp
            series = special.ive(0, A) + sum(2 * special.ive(k * N // 2, A) * math.cos(k * N * a / 2)
                                             for k in range(1, 40))
            ln = np.log(np.sum(q * series * np.exp(A - 0.5 * hh[0] * u * u)))
            assert r["lnl"][i, e] == pytest.approx(ln, abs=1e-9)


# ---------------------------------------------------------------- P5 ------
def test_distance_quadrature_converged(tiny):
    """The 2000-node rule agrees with 4000 nodes (Sec. IV B distance
    marginalisation computed to well below the 1e-3 target)."""
    wl = tiny.subset(rows=np.arange(4), cols=np.arange(16))
    r = O.eval_pairs_block(wl, np.arange(4), return_triples=True)
    a = O.ln_dist_marg(r["dh"], r["hh"], wl.d_max, wl.d0, 2000)
    b = O.ln_dist_marg(r["dh"], r["hh"], wl.d_max, wl.d0, 4000)
    assert np.max(np.abs(a - b)) < 1e-8
    # high SNR (50) peak is still resolved
    wl50 = W.config_tiny(seed=4, n_int=2, n_ext=2, snr=50.0, in_bank=True, noise_on=False)
    m = wl50.meta
    r = O.eval_pairs_block(wl50, [0], ext_idx=[0], return_triples=True)
    dh, hh = r["dh"][0, 0, m["inj_o"]], r["hh"][0, 0, m["inj_o"]]
    assert abs(O.ln_dist_marg(dh, hh, wl50.d_max, 1.0, 2000) - O.ln_dist_marg(dh, hh, wl50.d_max, 1.0, 5000)) < 1e-8


def test_laplace_asymptote():
    """At high SNR, ln Lbar -> lnL^ML + ln(pi(D*) sqrt(2 pi) sigma_D) with
    D* = d0 hh/dh and sigma_D = D*^2 / (d0 sqrt(hh)) (Laplace's method on
    eq. lnl_dist_marginalized)."""
    dmax, d0 = 5000.0, 1.0
    rho = 200.0
    for dstar in (300.0, 800.0, 2000.0):
        hh = (rho * dstar / d0) ** 2
        dh = hh * d0 / dstar
        sig = dstar ** 2 / (d0 * math.sqrt(hh))
        lap = dh * dh / (2 * hh) + math.log(3 * dstar ** 2 / dmax ** 3 * math.sqrt(2 * math.pi) * sig)
        got = float(O.ln_dist_marg(dh, hh, dmax, d0, 2000))
        assert got == pytest.approx(lap, abs=0.05)


# ---------------------------------------------------------------- P6 ------
def test_marginal_bounds(tiny):
    """Lbar <= exp(lnL^ML) (prior normalised, lnL(D) <= lnL^ML) and Jensen:
    ln Lbar >= dh E[u] - hh E[u^2]/2 under the rule's own weights."""
    wl = tiny.subset(rows=np.arange(4), cols=np.arange(32))
    r = O.eval_pairs_block(wl, np.arange(4), return_triples=True)
    dh, hh = r["dh"], r["hh"]
    lnl = O.ln_dist_marg(dh, hh, wl.d_max, wl.d0)
    assert np.all(lnl <= O.lnl_ml(dh, hh) + 1e-9)
    D, q = O.distance_nodes(wl.d_max)
    u = wl.d0 / D
    assert np.all(lnl >= dh * np.sum(q * u) - 0.5 * hh * np.sum(q * u * u) - 1e-9)


# ---------------------------------------------------------------- P7 ------
def test_residual_identity_against_simulator(tiny):
    """dh - hh/2 = [(d|d) - (d-h|d-h)]/2 (eq. lnlike), with h built by the
    independent forward simulator at (i, e, o, D = d0)."""
    wl = tiny
    net = W.Network(("H", "L"), wl.det_r, wl.det_D, np.ones(2))
    rng = np.random.default_rng(9)
    rows, cols = rng.choice(wl.n_int, 5, replace=False), rng.choice(wl.n_ext, 5, replace=False)
    r = O.eval_pairs_block(wl, rows, ext_idx=cols, return_triples=True)
    dd = O.data_inner(wl.d, wl.w)
    for a, i in enumerate(rows):
        for b, e in enumerate(cols):
            for o in (0, 5, 11):
                ext1 = {k: v[e] for k, v in wl.ext.items()}
                hk = W.simulate_strain(wl.h[i], wl.modes, wl.f, net, ext1, 2 * np.pi * o / wl.n_phi, wl.d0)
                rr = float(np.sum(wl.w * np.abs(wl.d - hk) ** 2))
                lhs = r["dh"][a, b, o] - 0.5 * r["hh"][a, b, o]
                assert lhs == pytest.approx(0.5 * (dd - rr), rel=1e-9, abs=1e-6 * dd)


def test_residual_identity_higher_modes():
    wl = W.config_production(seed=21, n_int=3, n_ext=3, snr=25.0)
    net = W.Network(("H", "L", "V"), wl.det_r, wl.det_D, np.ones(3))
    r = O.eval_pairs_block(wl, np.arange(3), return_triples=True)
    dd = O.data_inner(wl.d, wl.w)
    for i in range(3):
        for e in range(3):
            for o in (0, 7, 19):
                ext1 = {k: v[e] for k, v in wl.ext.items()}
                hk = W.simulate_strain(wl.h[i], wl.modes, wl.f, net, ext1, 2 * np.pi * o / wl.n_phi, wl.d0)
                rr = float(np.sum(wl.w * np.abs(wl.d - hk) ** 2))
                lhs = r["dh"][i, e, o] - 0.5 * r["hh"][i, e, o]
                assert lhs == pytest.approx(0.5 * (dd - rr), rel=1e-9, abs=1e-6 * dd)


# ---------------------------------------------------------------- P8 ------
def test_antenna_invariants():
    """eq. (response_plus/cross): F_+^2 + F_x^2 does not depend on psi;
    sky- and psi-averaged F_+^2 = 1/5 for a right-angle interferometer;
    overhead source: |F_+| = 1 at the arm-aligned psi; |t_k - t_geo| <= R/c."""
    net = W.network("HLV")
    rng = np.random.default_rng(1)
    n = 200000
    ext = W.draw_extrinsic(rng, n)
    F = O.antenna_patterns(net.D, ext["lat"], ext["lon"], ext["psi"])
    F2 = O.antenna_patterns(net.D, ext["lat"], ext["lon"], ext["psi"] + 0.7)
    assert np.allclose(F[..., 0] ** 2 + F[..., 1] ** 2, F2[..., 0] ** 2 + F2[..., 1] ** 2, atol=1e-12)
    mean = np.mean(F[..., 0] ** 2, axis=0)
    assert np.allclose(mean, 0.2, atol=4e-3)
    for k, name in enumerate("HLV"):
        lat, lon, az, _ = W.SITES[name]
        vals = [O.antenna_patterns(net.D[k:k + 1], [np.radians(lat)], [np.radians(lon)], [p])[0, 0]
                for p in np.linspace(0, np.pi, 721)]
        vals = np.array(vals)
        assert np.max(np.abs(vals[:, 0])) == pytest.approx(1.0, abs=1e-5)
        assert np.min(np.hypot(vals[:, 0], vals[:, 1])) == pytest.approx(1.0, abs=1e-9)
    t = O.arrival_times(net.r, ext["lat"], ext["lon"], ext["t_geo"])
    assert np.all(np.abs(t - ext["t_geo"][:, None]) <= W.EARTH_RADIUS_M / O.C_SI * (1 + 1e-12))


# ---------------------------------------------------------------- P9 ------
def test_swsh_orthonormal_and_closed_forms():
    """-2Y_lm: orthonormal on the sphere; (2,2) and (2,1) textbook forms."""
    x, wq = np.polynomial.legendre.leggauss(64)
    for m in range(-4, 5):
        ls = [l for l in range(2, 7) if l >= abs(m)]
        G = np.array([[2 * np.pi * np.sum(wq * O.swsh_m2(l1, m, x) * O.swsh_m2(l2, m, x))
                       for l2 in ls] for l1 in ls])
        assert np.allclose(G, np.eye(len(ls)), atol=1e-12)
    c = np.linspace(-1, 1, 11)
    s = np.sqrt(1 - c * c)
    assert np.allclose(O.swsh_m2(2, 2, c), math.sqrt(5 / (64 * math.pi)) * (1 + c) ** 2)
    assert np.allclose(O.swsh_m2(2, -2, c), math.sqrt(5 / (64 * math.pi)) * (1 - c) ** 2)
    assert np.allclose(O.swsh_m2(2, 1, c), math.sqrt(5 / (16 * math.pi)) * s * (1 + c))
    # (2,2) mode factors: K_+ = sqrt(5/64pi)(1+c^2), K_x = -2i sqrt(5/64pi) c
    K = O.mode_factors(((2, 2),), c)
    assert np.allclose(K[:, 0, 0], math.sqrt(5 / (64 * math.pi)) * (1 + c * c))
    assert np.allclose(K[:, 0, 1], -2j * math.sqrt(5 / (64 * math.pi)) * c)


# ---------------------------------------------------------------- P10 -----
def test_evidence_invariances(tiny):
    """eq. (Z_sum): permutations leave ln Z unchanged; duplicating the bank
    with N_norm doubled leaves it unchanged; w_i -> c w_i shifts it by ln c;
    a single pair gives Z = w_i w_e Lbar / (N_norm N_ext)."""
    rng = np.random.default_rng(2)
    lnl = rng.normal(0, 3, (7, 5))
    lwi, lwe = rng.normal(0, 1, 7), rng.normal(0, 1, 5)
    z = O.evidence_from_lnl(lnl, lwi, lwe)["ln_z"]
    p, q = rng.permutation(7), rng.permutation(5)
    assert O.evidence_from_lnl(lnl[p][:, q], lwi[p], lwe[q])["ln_z"] == pytest.approx(z, abs=1e-12)
    dup = O.evidence_from_lnl(np.vstack([lnl, lnl]), np.r_[lwi, lwi], lwe, n_norm=14)["ln_z"]
    assert dup == pytest.approx(z, abs=1e-12)
    assert O.evidence_from_lnl(lnl, lwi + 0.3, lwe)["ln_z"] == pytest.approx(z + 0.3, abs=1e-12)
    one = O.evidence_from_lnl(lnl[:1, :1], lwi[:1], lwe[:1], n_norm=10)["ln_z"]
    assert one == pytest.approx(lwi[0] + lwe[0] + lnl[0, 0] - math.log(10), abs=1e-12)
    # N_eff = (sum p)^2 / sum p^2 lies in [1, N] (eq. n_effective)
    ev = O.evidence_from_lnl(lnl, lwi, lwe)
    assert 1.0 <= ev["n_eff"] <= lnl.size


# ---------------------------------------------------------------- P11 -----
def test_time_shift_covariance(tiny):
    """Shifting the data by exp(-2 pi i f tau) and every t_geo by tau leaves
    all inner products unchanged (time-shift factor T of Sec. IV A)."""
    wl = tiny.subset(rows=np.arange(3), cols=np.arange(8))
    r0 = O.eval_pairs_block(wl, np.arange(3), return_triples=True)
    tau = 0.0123
    wl2 = wl.subset()
    wl2.d = wl.d * np.exp(-2j * np.pi * wl.f * tau)[None, :]
    wl2.ext = dict(wl.ext)
    wl2.ext["t_geo"] = wl.ext["t_geo"] + tau
    r1 = O.eval_pairs_block(wl2, np.arange(3), return_triples=True)
    assert np.allclose(r0["dh"], r1["dh"], rtol=1e-9, atol=1e-9 * np.max(np.abs(r0["dh"])))
    assert np.allclose(r0["lnl"], r1["lnl"], atol=1e-8)


# ---------------------------------------------------------------- P12 -----
def _brute_lnl(wl, i, e, n_nodes=2000):
    """Scalar loops over detectors, bins, channels, phases and distances."""
    lat, lon = wl.ext["lat"][e], wl.ext["lon"][e]
    psi, ci, tg = wl.ext["psi"][e], wl.ext["cos_iota"][e], wl.ext["t_geo"][e]
    n = (math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat))
    elon = (-math.sin(lon), math.cos(lon), 0.0)
    elat = (-math.sin(lat) * math.cos(lon), -math.sin(lat) * math.sin(lon), math.cos(lat))
    X = [math.cos(psi) * elon[a] + math.sin(psi) * elat[a] for a in range(3)]
    Y = [-math.sin(psi) * elon[a] + math.cos(psi) * elat[a] for a in range(3)]
    s = math.sqrt(1 - ci * ci)
    # textbook -2Y for l = 2
    Y2 = {2: math.sqrt(5 / (64 * math.pi)) * (1 + ci) ** 2, -2: math.sqrt(5 / (64 * math.pi)) * (1 - ci) ** 2,
          1: math.sqrt(5 / (16 * math.pi)) * s * (1 + ci), -1: math.sqrt(5 / (16 * math.pi)) * s * (1 - ci)}
    lse_terms = []
    for o in range(wl.n_phi):
        phi = 2 * math.pi * o / wl.n_phi
        dh = 0.0
        hh = 0.0
        for k in range(wl.d.shape[0]):
            Dk = wl.det_D[k]
            fp = sum(Dk[a][b] * (X[a] * X[b] - Y[a] * Y[b]) for a in range(3) for b in range(3))
            fx = sum(Dk[a][b] * (X[a] * Y[b] + Y[a] * X[b]) for a in range(3) for b in range(3))
            tk = tg - sum(wl.det_r[k][a] * n[a] for a in range(3)) / O.C_SI
            for bb in range(len(wl.f)):
                hv = 0j
                for c, (l, m) in enumerate(wl.modes):
                    kp = 0.5 * (Y2[-m] + Y2[m])
                    kx = 0.5j * (Y2[-m] - Y2[m])
                    hv += wl.h[i][c][bb] * (fp * kp + fx * kx) * cmath.exp(-1j * m * phi)
                hv *= cmath.exp(-2j * math.pi * wl.f[bb] * tk)
                dh += wl.w[k][bb] * (wl.d[k][bb] * hv.conjugate()).real
                hh += wl.w[k][bb] * abs(hv) ** 2
        terms = []
        xg, wg = np.polynomial.legendre.leggauss(n_nodes)
        Ds = [0.5 * wl.d_max * (float(x) + 1.0) for x in xg]
        norm = sum(float(wg[j]) * Ds[j] ** 2 for j in range(n_nodes))
        for j in range(n_nodes):
            D = Ds[j]
            terms.append(math.log(float(wg[j]) * D * D / norm) + dh * wl.d0 / D - 0.5 * hh * (wl.d0 / D) ** 2)
        mx = max(terms)
        lse_terms.append(mx + math.log(sum(math.exp(t - mx) for t in terms)))
    mx = max(lse_terms)
    return mx + math.log(sum(math.exp(t - mx) for t in lse_terms)) - math.log(wl.n_phi)


def test_brute_force_tiny():
    """All steps by scalar loops on a tiny problem (4 x 4 x 4 phases x 8 bins),
    22 + 21 modes (textbook l = 2 harmonics), random weights."""
    wl = W.make_workload(31, n_int=4, n_ext=4, n_bins=8, modes=((2, 2), (2, 1)), dets="HLV",
                         n_phi=4, snr=10.0, mc_range=(5.0, 15.0), q_range=(0.2, 0.6),
                         random_weights=True)
    r = O.eval_pairs_block(wl, np.arange(4))
    brute = np.array([[_brute_lnl(wl, i, e, 400) for e in range(4)] for i in range(4)])
    fast = O.eval_pairs_block(wl, np.arange(4), n_nodes=400)["lnl"]
    assert np.allclose(brute, fast, atol=1e-10, rtol=0)
    # evidence by loops
    tot = [wl.ln_w_int[i] + wl.ln_w_ext[e] + brute[i, e] for i in range(4) for e in range(4)]
    mx = max(tot)
    lnz = mx + math.log(sum(math.exp(t - mx) for t in tot)) - math.log(4) - math.log(4)
    assert O.evidence_from_lnl(fast, wl.ln_w_int, wl.ln_w_ext)["ln_z"] == pytest.approx(lnz, abs=1e-10)
    assert r["lnl"].shape == (4, 4)


def test_top_k_order():
    """Top-k: descending ln p, ties broken by (i, e) ascending."""
    lnp = np.array([[1.0, 3.0, 3.0], [3.0, 0.5, 2.0]])
    idx, vals = O.top_k(lnp, 4)
    assert idx.tolist() == [[0, 1], [0, 2], [1, 0], [1, 2]]
    assert vals.tolist() == [3.0, 3.0, 3.0, 2.0]


def test_zero_template_is_prior():
    """A template that vanishes in band (hh = 0) gives Lbar = 1."""
    assert float(O.ln_dist_marg(0.0, 0.0, 5000.0)) == pytest.approx(0.0, abs=1e-14)
    assert float(O.lnl_ml(0.0, 0.0)) == 0.0


# ------------------------------------------------------- P3 / P5 (sharp) ------
def test_adaptive_distance_rule_pins():
    """The adaptive-quadrature form of eq. (lnl_dist_marginalized), used
    where a fixed node set cannot resolve the peak, is pinned three ways:
    it equals the 2000-node Gauss-Legendre rule where that resolves the peak; with d = 0 it equals the closed form
    e^{-x0^2}(1 - 2 x0^2) + 2 sqrt(pi) x0^3 erfc(x0), x0 = (d0/D_max) sqrt(hh/2);
    and for sharp interior peaks it follows Laplace's expansion in
    u = d0/D: with z = dh/sqrt(hh) and u* = dh/hh, the u^-4 factor of the
    integrand averages to u*^-4 (1 + 10/z^2 + 105/z^4 + O(z^-6)) over the
    Gaussian peak of width u*/z."""
    dmax, d0 = 5000.0, 1.0
    for z, s in [(0.0, 1.0), (3.0, 2.0), (10.0, 5.0), (20.0, 3.0), (-5.0, 1.0), (0.5, 1e-3),
                 (40.0, 20.0), (8.0, 0.3)]:
        hh = (s * dmax / d0) ** 2
        dh = z * math.sqrt(hh)
        a = float(O.ln_dist_marg_adaptive(dh, hh, dmax, d0))
        assert a == pytest.approx(float(O.ln_dist_marg(dh, hh, dmax, d0, 2000)), abs=1e-10)
    # (the closed form cancels between its two terms as x0 grows: ~1e-11 at x0 = 20)
    for hh, tol in ((1e-2, 1e-12), (1.0, 1e-12), (1e4, 1e-12), ((2.0 * dmax) ** 2, 1e-11),
                    ((30.0 * dmax) ** 2, 1e-9)):
        x0 = (d0 / dmax) * math.sqrt(hh / 2.0)
        closed = math.exp(-x0 * x0) * ((1 - 2 * x0 * x0) + 2 * math.sqrt(math.pi) * x0 ** 3 * special.erfcx(x0))
        assert float(O.ln_dist_marg_adaptive(0.0, hh, dmax, d0)) == pytest.approx(math.log(closed), abs=tol)
    for z, dstar in [(30.0, 500.0), (60.0, 2.0), (60.0, 0.01), (200.0, 1000.0), (2000.0, 40.0)]:
        hh = (z * dstar / d0) ** 2          # peak at D* = d0 hh / dh
        dh = z * math.sqrt(hh)
        sig = dstar ** 2 / (d0 * math.sqrt(hh))
        lap = dh * dh / (2 * hh) + math.log(3 * dstar ** 2 / dmax ** 3 * math.sqrt(2 * math.pi) * sig)
        series = lap + math.log1p(10.0 / z ** 2 + 105.0 / z ** 4)
        got = float(O.ln_dist_marg_adaptive(dh, hh, dmax, d0))
        assert abs(got - series) < 2e3 / z ** 6 + 1e-11 * abs(got), (z, dstar, got - series)
    # a peak far narrower than the 2000-node spacing near D = 0: the fixed
    # rule is off by order one there, the adaptive one follows Laplace
    hh = (60.0 * 0.01) ** 2
    dh = 60.0 * math.sqrt(hh)
    assert abs(float(O.ln_dist_marg(dh, hh, dmax, d0, 2000)) - float(O.ln_dist_marg_adaptive(dh, hh, dmax, d0))) > 0.1


def test_eval_lnl_multiprocess_equals_single():
    """The oracle's multi-process split over bank rows returns the rows in
    order and bit-identical values (every row is computed by the same code
    on the same inputs, whichever process takes it)."""
    wl = W.config_production(seed=21, n_int=13, n_ext=24, n_bins=64, random_weights=True)
    one = O.eval_lnl(wl, processes=1)
    two = O.eval_lnl(wl, processes=2)
    assert np.array_equal(one["lnl"], two["lnl"])
    assert np.array_equal(one["ml_max"], two["ml_max"])
    # and the rows are in bank order: row i equals a one-row evaluation of row i
    for i in (0, 6, 12):
        r = O.eval_pairs_block(wl, [i])
        assert np.array_equal(r["lnl"][0], one["lnl"][i])
