"""FP64 CPU oracle for the likelihood-matrix hot path -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
use this module.  It is the plain definition of what the hot path computes,
written from the paper (arXiv:2507.16022) without any of the GPU path's
rearrangements: every (waveform i, extrinsic sample e, phase o) triple gets
its own detector waveform, its inner products are direct sums over all
frequency bins, distance is integrated with 2000-node Gauss-Legendre and
the evidence is a log-sum-exp over all pairs.  It shares no code with the
GPU library and does not import it.

Readings of the paper (where it is silent, ambiguous or garbled):
  * the distance-marginalised likelihood of eq. (lnl_dist_marginalized) is
    the integral itself (the "ln" on its left-hand side is a typo);
  * the (h|h) inner product of eq. (hh_ieo) is per detector with that
    detector's noise weights;
  * modes are (l, m) channels; the orbital-phase factor uses m of the
    channel, applied as exp(-i m phi) to the waveform (sign immaterial on
    a regular phase grid, which maps o -> N-o);
  * arrival time t_k = t_geo - r_k . n / c with n pointing to the source;
  * inner products are sums over the given frequency bins with weights
    w_kb = 4 df_b / S_k(f_b) (relative-binning summaries with
    W^{dh} = w d and W^{hh} = w on those bins);
  * non-precessing waveforms: the inclination dependence factorises into
    K_{c,p}(iota), so the bank stores one complex amplitude per (l, m) and
    the inclination travels with the extrinsic sample;
  * phase grid phi_o = 2 pi o / N_phi, w_o = 1 (Sec. IV B);
  * distance prior proportional to D^2 on (0, D_max].
"""
from __future__ import annotations

import functools
import math

import numpy as np

C_SI = 299792458.0


def _lse(x, axis=-1):
    """log(sum(exp(x))) along an axis, stable; -inf for all -inf input."""
    x = np.asarray(x, dtype=np.float64)
    m = np.max(x, axis=axis, keepdims=True)
    m_safe = np.where(np.isfinite(m), m, 0.0)
    s = np.sum(np.exp(x - m_safe), axis=axis, keepdims=True)
    out = np.log(s) + m_safe
    return np.squeeze(out, axis=axis)


# --------------------------------------------------------------------------
# O1: geometry -- eq. (thetaext), (response_plus/cross), (t_at_detector)
# --------------------------------------------------------------------------
def sky_direction(lat, lon):
    """Unit vector towards the source in the Earth-fixed frame, [N, 3]."""
    lat = np.asarray(lat, dtype=np.float64)
    lon = np.asarray(lon, dtype=np.float64)
    return np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)], -1)


def polarization_tensors(lat, lon, psi):
    """e_+ and e_x [N, 3, 3] for waves from (lat, lon) at polarisation psi.

    Transverse basis: X = cos(psi) e_lon + sin(psi) e_lat and
    Y = -sin(psi) e_lon + cos(psi) e_lat, with e_lon, e_lat the unit
    vectors of increasing longitude and latitude at the source direction.
    """
    lat, lon, psi = (np.asarray(a, dtype=np.float64) for a in (lat, lon, psi))
    e_lon = np.stack([-np.sin(lon), np.cos(lon), np.zeros_like(lon)], -1)
    e_lat = np.stack([-np.sin(lat) * np.cos(lon), -np.sin(lat) * np.sin(lon), np.cos(lat)], -1)
    X = np.cos(psi)[:, None] * e_lon + np.sin(psi)[:, None] * e_lat
    Y = -np.sin(psi)[:, None] * e_lon + np.cos(psi)[:, None] * e_lat
    ep = X[:, :, None] * X[:, None, :] - Y[:, :, None] * Y[:, None, :]
    ex = X[:, :, None] * Y[:, None, :] + Y[:, :, None] * X[:, None, :]
    return ep, ex


def antenna_patterns(det_D, lat, lon, psi):
    """F_{ekp}: [N_e, K, 2] real (p = +, x), the contraction D_k : e_p."""
    ep, ex = polarization_tensors(lat, lon, psi)
    fp = np.einsum("kab,eab->ek", det_D, ep)
    fx = np.einsum("kab,eab->ek", det_D, ex)
    return np.stack([fp, fx], -1)


def arrival_times(det_r, lat, lon, t_geo):
    """t_{ek} = t_geo - r_k . n / c  [N_e, K] (reading of eq. t_at_detector)."""
    n = sky_direction(lat, lon)
    return np.asarray(t_geo, dtype=np.float64)[:, None] - (n @ np.asarray(det_r).T) / C_SI


# --------------------------------------------------------------------------
# O2/O3: mode factors and complex response
# --------------------------------------------------------------------------
def swsh_m2(l, m, cos_t):
    """Spin-weight -2 spherical harmonic at azimuth 0, from the Wigner small-d
    matrix: -2Y_lm(theta, 0) = sqrt((2l+1)/(4 pi)) d^l_{m,2}(theta)."""
    cos_t = np.asarray(cos_t, dtype=np.float64)
    th = np.arccos(np.clip(cos_t, -1.0, 1.0))
    cb, sb = np.cos(th / 2), np.sin(th / 2)
    j, mp, mm = l, m, 2          # d^j_{m' m}: m' = m (mode), m = 2 (spin)
    fac = math.factorial
    out = np.zeros_like(cos_t)
    for k in range(0, 2 * j + 1):
        a, b, c, d = j + mm - k, k, j - k - mp, k - mm + mp
        if min(a, b, c, d) < 0:
            continue
        coef = (-1.0) ** (k - mm + mp) * math.sqrt(fac(j + mm) * fac(j - mm) * fac(j + mp) * fac(j - mp)) \
            / (fac(a) * fac(b) * fac(c) * fac(d))
        out = out + coef * cb ** (2 * j - 2 * k + mm - mp) * sb ** (2 * k - mm + mp)
    return math.sqrt((2 * l + 1) / (4 * math.pi)) * out


def mode_factors(modes, cos_iota):
    """K_{c,p}(iota): [N_e, N_c, 2] complex.  For a non-precessing source the
    positive-frequency + and x polarisations of channel (l, m) are
    K_+ = (Y_{l,-m} + (-1)^l Y_{lm})/2 and K_x = i (Y_{l,-m} - (-1)^l Y_{lm})/2
    times the stored mode amplitude."""
    out = np.zeros((len(cos_iota), len(modes), 2), dtype=np.complex128)
    for c, (l, m) in enumerate(modes):
        yn = swsh_m2(l, -m, cos_iota)
        yp = swsh_m2(l, m, cos_iota)
        out[:, c, 0] = 0.5 * (yn + (-1) ** l * yp)
        out[:, c, 1] = 0.5j * (yn - (-1) ** l * yp)
    return out


def response(wl_det_D, modes, ext):
    """R_{ekc} = sum_p F_{ekp} K_{cp}(iota_e): [N_e, K, N_c] complex."""
    F = antenna_patterns(wl_det_D, ext["lat"], ext["lon"], ext["psi"])
    Kf = mode_factors(modes, ext["cos_iota"])
    return np.einsum("ekp,ecp->ekc", F.astype(np.complex128), Kf)


# --------------------------------------------------------------------------
# O4/O5: detector waveforms and inner products, per triple, direct sums
# --------------------------------------------------------------------------
def phase_grid(n_phi):
    return 2.0 * np.pi * np.arange(n_phi) / n_phi


def triple_inner_products(h_i, R, t, f, mode_m, phis, d, w):
    """dh, hh for one waveform against a block of extrinsic samples.

    h_i [N_c, N_b]; R [E, K, N_c]; t [E, K]; returns dh, hh [E, N_phi].
    h_{eokb} = sum_c h_{cb} R_{ekc} exp(-2 pi i f_b t_{ek}) exp(-i m_c phi_o)
    (eq. h_k at d0), dh = Re sum_kb w d conj(h), hh = sum_kb w |h|^2
    (eq. inner_product).
    """
    T = np.exp(-2j * np.pi * f[None, None, :] * t[:, :, None])          # [E,K,B]
    Phi = np.exp(-1j * np.outer(phis, mode_m))                          # [O,C]
    hk = np.einsum("cb,ekc,oc->eokb", h_i, R, Phi) * T[:, None, :, :]  # [E,O,K,B]
    dh = np.real(np.einsum("kb,eokb->eo", w * d, np.conj(hk)))
    hh = np.einsum("kb,eokb->eo", w, np.abs(hk) ** 2)
    return dh, hh


def data_inner(d, w):
    """(d|d) = sum_kb w |d|^2."""
    return float(np.sum(w * np.abs(d) ** 2))


# --------------------------------------------------------------------------
# O6/O7: maximum likelihood over distance, distance marginalisation
# --------------------------------------------------------------------------
def lnl_at_distance(dh, hh, dist, d0=1.0):
    """eq. (lnlike_ieo_arb_dL)."""
    x = dist / d0
    return dh / x - 0.5 * hh / x ** 2


def lnl_ml(dh, hh):
    """eq. (bestfit_lnl): dh^2/(2 hh) if dh > 0 else 0."""
    dh = np.asarray(dh, dtype=np.float64)
    hh = np.asarray(hh, dtype=np.float64)
    pos = dh > 0
    out = np.zeros(np.broadcast(dh, hh).shape)
    np.divide(dh * dh, 2.0 * hh, out=out, where=pos & (hh > 0))
    return out


@functools.lru_cache(maxsize=8)
def _gl(n_nodes):
    return np.polynomial.legendre.leggauss(n_nodes)


def distance_nodes(d_max, n_nodes=2000):
    """Gauss-Legendre nodes D_j on (0, D_max] and normalised weights q_j for
    the prior proportional to D^2 (q_j proportional to GL weight x D_j^2,
    summing to one)."""
    x, wq = _gl(int(n_nodes))
    D = 0.5 * d_max * (x + 1.0)
    q = wq * D * D
    return D, q / np.sum(q)


def ln_dist_marg(dh, hh, d_max, d0=1.0, n_nodes=2000, chunk=4096):
    """ln of eq. (lnl_dist_marginalized): ln sum_j q_j exp(dh u_j - hh u_j^2/2),
    2000-node Gauss-Legendre in D over (0, D_max] (the integrand vanishes
    smoothly at D -> 0 and is cut hard at D_max, where a Gauss rule keeps
    its accuracy), 
    u_j = d0/D_j, evaluated in log space.  dh, hh: arrays of equal shape."""
    dh = np.asarray(dh, dtype=np.float64)
    hh = np.asarray(hh, dtype=np.float64)
    shape = np.broadcast(dh, hh).shape
    dh = np.broadcast_to(dh, shape).ravel()
    hh = np.broadcast_to(hh, shape).ravel()
    D, q = distance_nodes(d_max, n_nodes)
    u = d0 / D
    lq = np.log(q)
    out = np.empty(dh.shape)
    for s in range(0, dh.size, chunk):
        a = dh[s:s + chunk, None]
        b = hh[s:s + chunk, None]
        out[s:s + chunk] = _lse(lq[None, :] + a * u[None, :] - 0.5 * b * (u * u)[None, :], axis=1)
    return out.reshape(shape)


def ln_dist_marg_adaptive(dh, hh, d_max, d0=1.0, rel=1e-12):
    """ln of eq. (lnl_dist_marginalized) by adaptive quadrature (scipy's
    quad), for peaks narrower than a fixed node set resolves.

    With u = d0/D the prior D^2 on (0, D_max] turns the integral into
    3 u0^3 int_{u0}^inf u^-4 exp(dh u - hh u^2/2) du, u0 = d0/D_max.  The
    exponent's largest value over u >= u0 (at u* = max(u0, dh/hh)) is taken
    out, and [u0, u* + 40/sqrt(hh)] is cut into pieces that quad integrates
    separately: doubling steps from u0 (where u^-4 changes on the scale u0)
    and steps of one peak width 1/sqrt(hh) around u*.  Past the last piece
    the integrand is below exp(-800) of its peak."""
    import warnings

    from scipy import integrate
    dh = np.asarray(dh, dtype=np.float64)
    hh = np.asarray(hh, dtype=np.float64)
    dh, hh = np.broadcast_arrays(dh, hh)
    out = np.empty(dh.shape)
    u0 = d0 / d_max
    for idx in np.ndindex(dh.shape):
        a, b = float(dh[idx]), float(hh[idx])
        if not b > 0.0:
            if a == 0.0:
                out[idx] = 0.0          # empty template: the prior integrates to one
                continue
            raise ValueError("hh must be positive unless dh = 0")
        sig = 1.0 / math.sqrt(b)
        ustar = max(u0, a / b)
        c = a * ustar - 0.5 * b * ustar * ustar
        hi = ustar + 40.0 * sig
        pts = {u0, hi}
        u = u0
        while u < hi:
            pts.add(u)
            u *= 2.0
        for k in range(-40, 41):
            x = ustar + k * sig
            if u0 < x < hi:
                pts.add(x)
        pts = sorted(pts)

        def f(u):
            return u ** -4 * math.exp(a * u - 0.5 * b * u * u - c)

        tot = 0.0
        with warnings.catch_warnings():
            # quad flags pieces whose share is below the rounding of the sum
            warnings.simplefilter("ignore", integrate.IntegrationWarning)
            for lo, up in zip(pts[:-1], pts[1:]):
                tot += integrate.quad(f, lo, up, epsabs=0.0, epsrel=rel, limit=200)[0]
        out[idx] = math.log(3.0) + 3.0 * math.log(u0) + c + math.log(tot)
    return out


# --------------------------------------------------------------------------
# O8-O10: per-pair likelihood, evidence, top-K
# --------------------------------------------------------------------------
def eval_pairs_block(wl, rows, ext_idx=None, n_nodes=2000, return_triples=False,
                     return_phase=False):
    """ln Lbar_ie for bank rows `rows` x extrinsic samples `ext_idx`.

    Returns dict with lnl [len(rows), E] and max lnL^ML [len(rows), E];
    with return_triples also dh, hh [len(rows), E, N_phi]; with
    return_phase also lnl_phase [len(rows), E, N_phi], the distance-
    marginalised ln Lbar_ieo of each triple.
    """
    ext_idx = np.arange(wl.n_ext) if ext_idx is None else np.asarray(ext_idx)
    ext = {k: np.asarray(v)[ext_idx] for k, v in wl.ext.items()}
    R = response(wl.det_D, wl.modes, ext)
    t = arrival_times(wl.det_r, ext["lat"], ext["lon"], ext["t_geo"])
    phis = phase_grid(wl.n_phi)
    mode_m = np.array([m for _, m in wl.modes], dtype=np.float64)
    E = len(ext_idx)
    lnl = np.empty((len(rows), E))
    mlmax = np.empty((len(rows), E))
    dhs = np.empty((len(rows), E, wl.n_phi)) if return_triples else None
    hhs = np.empty((len(rows), E, wl.n_phi)) if return_triples else None
    lph = np.empty((len(rows), E, wl.n_phi)) if return_phase else None
    eb = max(1, min(E, 262144 // max(1, wl.n_phi * wl.d.shape[0] * len(wl.f))))
    for a, i in enumerate(rows):
        for s in range(0, E, eb):
            sl = slice(s, s + eb)
            dh, hh = triple_inner_products(wl.h[i], R[sl], t[sl], wl.f, mode_m, phis, wl.d, wl.w)
            lnl_o = ln_dist_marg(dh, hh, wl.d_max, wl.d0, n_nodes)
            lnl[a, sl] = _lse(lnl_o, axis=1) - math.log(wl.n_phi)
            if return_phase:
                lph[a, sl] = lnl_o
            mlmax[a, sl] = np.max(lnl_ml(dh, hh), axis=1)
            if return_triples:
                dhs[a, sl] = dh
                hhs[a, sl] = hh
    out = dict(lnl=lnl, ml_max=mlmax)
    if return_triples:
        out.update(dh=dhs, hh=hhs)
    if return_phase:
        out.update(lnl_phase=lph)
    return out


def _worker(args):
    wl, rows, n_nodes = args
    return eval_pairs_block(wl, rows, None, n_nodes)


def eval_lnl(wl, n_nodes=2000, processes=1):
    """ln Lbar_ie for every bank row and extrinsic sample of the workload."""
    rows = np.arange(wl.n_int)
    if processes <= 1:
        return eval_pairs_block(wl, rows, None, n_nodes)
    import multiprocessing as mp
    import os
    chunks = [c for c in np.array_split(rows, processes * 4) if len(c)]
    ctx = mp.get_context("spawn")
    # one thread per worker process: the workers share the cores, and
    # numpy's threaded kernels in each of them would oversubscribe them
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "1" for k in keys})
    try:
        with ctx.Pool(processes) as pool:
            parts = pool.map(_worker, [(wl, c, n_nodes) for c in chunks])
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return dict(lnl=np.concatenate([p["lnl"] for p in parts]),
                ml_max=np.concatenate([p["ml_max"] for p in parts]))


def evidence_from_lnl(lnl, ln_w_int, ln_w_ext, n_norm=0.0):
    """eq. (Z_sum) with w_o = 1: ln Z = LSE_ie(ln w_i + ln w_e + ln Lbar_ie)
    - ln N_norm - ln N_ext.  Also ln sum p, ln sum p^2 (eq. n_effective)."""
    lnp = np.asarray(ln_w_int)[:, None] + np.asarray(ln_w_ext)[None, :] + lnl
    n_norm = float(n_norm) if n_norm and n_norm > 0 else float(lnl.shape[0])
    ln_sum_p = float(_lse(lnp.ravel()))
    ln_sum_p2 = float(_lse(2.0 * lnp.ravel()))
    ln_z = ln_sum_p - math.log(n_norm) - math.log(lnl.shape[1])
    return dict(ln_z=ln_z, ln_sum_p=ln_sum_p, ln_sum_p2=ln_sum_p2,
                n_eff=math.exp(2 * ln_sum_p - ln_sum_p2), lnp=lnp)


def top_k(lnp, k):
    """Top-k (i, e) pairs by ln p descending, ties by i then e ascending."""
    n_i, n_e = lnp.shape
    flat = lnp.ravel()
    order = np.lexsort((np.arange(flat.size), -flat))   # stable: index order
    sel = order[:k]
    return np.stack([sel // n_e, sel % n_e], -1), flat[sel]


def evidence(wl, n_nodes=2000, processes=1, k=0):
    """Full oracle: ln Z, N_eff ingredients, max lnL^ML, (d|d), top-k."""
    r = eval_lnl(wl, n_nodes, processes)
    ev = evidence_from_lnl(r["lnl"], wl.ln_w_int, wl.ln_w_ext, wl.n_norm)
    out = dict(ln_z=ev["ln_z"], ln_sum_p=ev["ln_sum_p"], ln_sum_p2=ev["ln_sum_p2"],
               n_eff=ev["n_eff"], max_lnl_ml=float(np.max(r["ml_max"])),
               dd=data_inner(wl.d, wl.w), lnl=r["lnl"], lnp=ev["lnp"])
    if k:
        idx, vals = top_k(ev["lnp"], k)
        out.update(topk_idx=idx, topk_lnp=vals)
    return out


# --------------------------------------------------------------------------
# O11: effective sample sizes (Sec. III B eq. n_effective; Sec. V A eqs.
# posterior_element, int_ess, ext_ess)
# --------------------------------------------------------------------------
def posterior_weights(wl, n_nodes=2000):
    """ln p_ieo = ln w_i + ln w_e + ln w_o + ln Lbar_ieo with w_o = 1/N_phi
    (eq. posterior_element): [N_i, N_e, N_phi]."""
    r = eval_pairs_block(wl, np.arange(wl.n_int), n_nodes=n_nodes, return_phase=True)
    return (np.asarray(wl.ln_w_int)[:, None, None] + np.asarray(wl.ln_w_ext)[None, :, None]
            + r["lnl_phase"] - math.log(wl.n_phi))


def effective_sizes(lnp3):
    """From ln p_ieo [N_i, N_e, N_phi]: N_eff over triples (eq.
    posterior_element), over intrinsic samples (eq. int_ess: squares of the
    row sums over e and o), over extrinsic samples (eq. ext_ess: squares of
    the column sums over i and o), and over pairs (eq. n_effective with
    p_ie = sum_o p_ieo)."""
    lnp3 = np.asarray(lnp3, dtype=np.float64)
    with np.errstate(divide="ignore"):      # rows or columns with no weight at all
        return _effective_sizes(lnp3)


def _effective_sizes(lnp3):
    tot = float(_lse(lnp3.ravel()))

    def ratio(ln_parts):
        return math.exp(2.0 * tot - float(_lse(2.0 * np.ravel(ln_parts))))

    rows = _lse(lnp3.reshape(lnp3.shape[0], -1), axis=1)
    cols = _lse(np.moveaxis(lnp3, 1, 0).reshape(lnp3.shape[1], -1), axis=1)
    pairs = _lse(lnp3, axis=2)
    return dict(n_eff=ratio(lnp3), n_eff_int=ratio(rows), n_eff_ext=ratio(cols),
                n_eff_pairs=ratio(pairs))


# --------------------------------------------------------------------------
# O12: posterior samples (Sec. III B: resampling by the probabilistic
# weights; Sec. V B: N_s = N_eff / 2)
# --------------------------------------------------------------------------
def splitmix64_uniform(seed, n):
    """Output n (from 0) of a SplitMix64 generator (Steele, Lea and Flood,
    2014) seeded with `seed`, as a uniform number in [0, 1) from its top 53
    bits."""
    mask = (1 << 64) - 1
    z = (int(seed) + (int(n) + 1) * 0x9E3779B97F4A7C15) & mask
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
    z ^= z >> 31
    return (z >> 11) * 2.0 ** -53


def systematic_draws(weights, n_s, u0):
    """Systematic resampling: draw s lands at cumulative mass (s + u0) W / n_s
    of the weights in the order given (W their total); returns the index of
    the first weight whose running sum exceeds it."""
    cum = np.cumsum(np.asarray(weights, dtype=np.float64))
    t = (np.arange(n_s) + u0) * cum[-1] / n_s
    return np.minimum(np.searchsorted(cum, t, side="right"), len(cum) - 1)


def inverse_cdf_index(weights, u):
    """The first index whose running sum of the weights exceeds u x total."""
    cum = np.cumsum(np.asarray(weights, dtype=np.float64))
    return int(min(np.searchsorted(cum, u * cum[-1], side="right"), len(cum) - 1))


def distance_posterior_draw(dh, hh, d_max, d0, u):
    """The distance drawn at the uniform number u from the posterior of eq.
    (lnl_dist_marginalized)'s integrand, pi(D) proportional to D^2 on
    (0, D_max]: in v = d0/D its density is proportional to
    v^-4 exp(dh v - hh v^2 / 2) on [d0/D_max, inf), and D = d0/v with
    P(v' <= v) = u (so P(D' >= D) = u).  The distribution function by
    adaptive quadrature, inverted by bisection to a relative 1e-12 in v."""
    from scipy import integrate, optimize
    v0 = d0 / d_max
    vs = max(v0, dh / hh) if hh > 0 else v0
    sg = 1.0 / math.sqrt(hh) if hh > 0 else v0
    c = max(-4.0 * math.log(v) + dh * v - 0.5 * hh * v * v for v in (v0, vs))

    def f(v):
        return math.exp(-4.0 * math.log(v) + dh * v - 0.5 * hh * v * v - c)

    # pieces: doubling steps from v0, and widths around the peak
    hi = max(vs + 40.0 * sg, 1e4 * v0)
    pts = {v0, hi}
    v = v0
    while v < hi:
        pts.add(v)
        v *= 2.0
    for k in range(-40, 41):
        x = vs + k * sg
        if v0 < x < hi:
            pts.add(x)
    pts = sorted(pts)
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        seg = [integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-12, limit=200)[0]
               for a, b in zip(pts[:-1], pts[1:])]
        total = sum(seg)
        target = u * total
        run = 0.0
        for (a, b), m in zip(zip(pts[:-1], pts[1:]), seg):
            if run + m >= target:
                g = lambda x: run + integrate.quad(f, a, x, epsabs=0.0, epsrel=1e-12, limit=200)[0] - target
                vv = optimize.brentq(g, a, b, xtol=1e-15, rtol=1e-12)
                return d0 / vv
            run += m
    return d0 / pts[-1]


# --------------------------------------------------------------------------
# P1: intrinsic pre-selection by the incoherent single-detector maximum
# likelihood (Sec. IV D; App. B eqs. dh_itop, x_ML, single_det_ML)
# --------------------------------------------------------------------------
def polarisations(h_i, modes, cos_iota, phis):
    """h_p(f) of one bank row at each grid phase: [N_phi, 2, N_b] complex,
    h_p = sum_c K_{c,p}(iota) h_c(f) exp(-i m_c phi) (p = +, x).  For the
    pre-selection the inclination is a property of the bank row."""
    K = mode_factors(modes, np.array([cos_iota], dtype=np.float64))[0]     # [C, 2]
    m = np.array([mm for _, mm in modes], dtype=np.float64)
    Phi = np.exp(-1j * np.outer(phis, m))                                  # [O, C]
    return np.einsum("cp,oc,cb->opb", K, Phi, np.asarray(h_i))


def _pinv_sym2(H, rel=1e-10):
    """Moore-Penrose pseudo-inverse of a real symmetric 2x2 matrix: its
    eigen-directions with eigenvalue below rel x the largest are dropped."""
    lam, V = np.linalg.eigh(H)
    top = np.max(np.abs(lam))
    out = np.zeros((2, 2))
    for q in range(2):
        if top > 0.0 and lam[q] > rel * top:
            out += np.outer(V[:, q], V[:, q]) / lam[q]
    return out


def single_detector_ml(h_i, modes, cos_iota, f, d_k, w_k, times, n_phi):
    """ln L^ML_{i k o t} of eq. (single_det_ML) for one bank row and one
    detector on the grid phase_grid(n_phi) x times: [N_phi, N_t].

    The detector's response and the distance become one free real
    amplitude per polarisation, x_p (eq. x_ML).  With
    b_p(o, t) = (d | h_p e^{-2 pi i f t}) (eq. dh_itop) and
    H_pp'(o) = (h_p | h_p') the largest ln L over x is b^T H^+ b / 2, H^+
    the pseudo-inverse (a polarisation that vanishes, as h_x does for an
    edge-on source, adds nothing)."""
    hp = polarisations(h_i, modes, cos_iota, phase_grid(n_phi))          # [O, 2, B]
    f = np.asarray(f, dtype=np.float64)
    shift = np.exp(2j * np.pi * np.outer(np.asarray(times, dtype=np.float64), f))   # [T, B]
    b = np.real(np.einsum("b,opb,tb->otp", np.asarray(w_k) * np.asarray(d_k), np.conj(hp), shift))
    H = np.real(np.einsum("b,opb,oqb->opq", np.asarray(w_k), hp, np.conj(hp)))
    out = np.empty((n_phi, len(times)))
    for o in range(n_phi):
        out[o] = 0.5 * np.einsum("tp,pq,tq->t", b[o], _pinv_sym2(H[o]), b[o])
    return out


def incoherent_ml(h, modes, cos_iota, f, d, w, t0, dt, n_t, n_phi):
    """ln L^{inco ML}_i = sum_k max_{o,t} ln L^ML_{ikot} (Sec. IV D) for the
    rows of h [N_rows, N_c, N_b]; detector k's time grid is
    t0[k] + j dt, j < n_t.  Returns (per row [N_rows], per row and detector
    [N_rows, K])."""
    n_rows, n_det = len(h), len(d)
    per = np.empty((n_rows, n_det))
    for i in range(n_rows):
        for k in range(n_det):
            times = t0[k] + dt * np.arange(n_t)
            per[i, k] = np.max(single_detector_ml(h[i], modes, cos_iota[i], f, d[k], w[k], times, n_phi))
    return per.sum(axis=1), per


def preselect(lnl_inco, delta=20.0):
    """Sec. IV D: the rows whose incoherent maximum likelihood is within
    delta of the largest (ascending row order)."""
    lnl_inco = np.asarray(lnl_inco)
    return np.flatnonzero(lnl_inco >= np.max(lnl_inco) - delta)


# --------------------------------------------------------------------------
# O13: the paper's own layout and relative binning (Sec. IV A eq. h_k with
# (m, p) channels and real F_kp; App. A eqs. dh_weights, hh_weights, d_h,
# h_h)
# --------------------------------------------------------------------------
def response_mp(det_D, pols, ext):
    """R_{ekc} = F_{ek,p_c} for channels c = (m_c, p_c), p = 0 (+) or 1 (x):
    the real antenna patterns of eq. (response_plus/cross) with the
    inclination inside the bank's h_{mp} (eq. thetaint), [N_e, K, N_c]."""
    F = antenna_patterns(det_D, ext["lat"], ext["lon"], ext["psi"])
    return F[:, :, np.asarray(pols, dtype=int)].astype(np.complex128)


def hat_splines(f, nodes):
    """s_b(f) [B, F]: the piecewise-linear functions on the nodes with
    s_b(f_b') = delta_bb', zero outside [f_0, f_{B-1}]."""
    f = np.asarray(f, dtype=np.float64)
    nodes = np.asarray(nodes, dtype=np.float64)
    s = np.zeros((len(nodes), len(f)))
    for b in range(len(nodes)):
        if b > 0:
            m = (f >= nodes[b - 1]) & (f <= nodes[b])
            s[b, m] = (f[m] - nodes[b - 1]) / (nodes[b] - nodes[b - 1])
        if b + 1 < len(nodes):
            m = (f >= nodes[b]) & (f <= nodes[b + 1])
            s[b, m] = (nodes[b + 1] - f[m]) / (nodes[b + 1] - nodes[b])
        s[b, f == nodes[b]] = 1.0
    return s


def rb_weights(f_full, d_full, w_full, h0, node_idx, t0=None):
    """Relative-binning weights (App. A) with <a|b>_k = sum_f w_kf a conj(b)
    over the full-resolution grid and the reference channel of detector k
    h0_kc(f) = h0_c(f) exp(-2 pi i f t0_k) (its arrival time; the one part of
    the reference's extrinsic parameters that does not cancel):
        W^dh_{kcb}   = <d_k | h0_kc s_b> / conj(h0_kc(f_b))              (eq. dh_weights)
        W^hh_{kcc'b} = <h0_kc | h0_kc' s_b> / (h0_kc(f_b) conj(h0_kc'(f_b)))  (eq. hh_weights)
    f_full [F]; d_full [K, F]; w_full [K, F]; h0 [C, F]; node_idx [B]
    indices of the spline nodes f_b in f_full; t0 [K] (None: 0).
    Returns W_dh [K, C, B], W_hh [K, C, C, B] (complex) and (d|d)."""
    f_full = np.asarray(f_full, dtype=np.float64)
    K = np.asarray(d_full).shape[0]
    t0 = np.zeros(K) if t0 is None else np.asarray(t0, dtype=np.float64)
    s = hat_splines(f_full, f_full[node_idx])
    h0k = np.asarray(h0, dtype=np.complex128)[None] * np.exp(-2j * np.pi * f_full[None, None, :]
                                                             * t0[:, None, None])   # [K,C,F]
    h0b = h0k[:, :, node_idx]
    wd = np.asarray(w_full) * np.asarray(d_full)
    W_dh = np.einsum("kf,kcf,bf->kcb", wd, np.conj(h0k), s) / np.conj(h0b)
    W_hh = np.einsum("kf,kcf,kdf,bf->kcdb", np.asarray(w_full, dtype=np.complex128), h0k,
                     np.conj(h0k), s) / (h0b[:, :, None, :] * np.conj(h0b)[:, None, :, :])
    dd = float(np.sum(np.asarray(w_full) * np.abs(d_full) ** 2))
    return W_dh, W_hh, dd


def triple_inner_products_rb(h_i, R, t, f, mode_m, phis, W_dh, W_hh):
    """dh, hh [E, N_phi] of one waveform with relative-binning weights:
    with h_{eokcb} = h_{cb} R_{ekc} exp(-2 pi i f_b t_{ek}) exp(-i m_c phi_o),
    dh = Re sum_{kcb} W^dh_{kcb} conj(h_{eokcb}) (eq. d_h) and
    hh = sum_{kcc'b} W^hh_{kcc'b} h_{eokcb} conj(h_{eokc'b}) (eq. h_h)."""
    T = np.exp(-2j * np.pi * np.asarray(f)[None, None, :] * t[:, :, None])       # [E,K,B]
    Phi = np.exp(-1j * np.outer(phis, mode_m))                                  # [O,C]
    hk = np.einsum("cb,ekc,oc->eokcb", h_i, R, Phi) * T[:, None, :, None, :]   # [E,O,K,C,B]
    dh = np.real(np.einsum("kcb,eokcb->eo", W_dh, np.conj(hk)))
    hh = np.real(np.einsum("kcdb,eokcb,eokdb->eo", W_hh, hk, np.conj(hk), optimize=True))
    return dh, hh


def eval_pairs_general(h, mode_m, R, t, f, n_phi, W_dh, W_hh, ln_w_int, ln_w_ext, d_max, d0,
                       n_nodes=2000):
    """Per pair ln Lbar_ie, max lnL^ML and per triple dh, hh for a bank h [N_i,
    C, B] against extrinsic responses R [E, K, C] and delays t [E, K], with
    relative-binning weights (plain bins: W_dh = w d, W_hh = w for every
    channel pair).  The rest as eval_pairs_block: eq. (lnl_dist_marginalized)
    by the 2000-node rule, the phase average, and ln p = ln w_i + ln w_e +
    ln Lbar."""
    phis = phase_grid(n_phi)
    n_i, E = h.shape[0], R.shape[0]
    lnl = np.empty((n_i, E))
    ml = np.empty((n_i, E))
    dhs = np.empty((n_i, E, n_phi))
    hhs = np.empty((n_i, E, n_phi))
    K, C, B = R.shape[1], R.shape[2], len(f)
    eb = max(1, (1 << 21) // (n_phi * K * C * B))      # extrinsic samples per block
    for i in range(n_i):
        for s in range(0, E, eb):
            sl = slice(s, s + eb)
            dh, hh = triple_inner_products_rb(h[i], R[sl], t[sl], f, mode_m, phis, W_dh, W_hh)
            lnl[i, sl] = _lse(ln_dist_marg(dh, hh, d_max, d0, n_nodes), axis=1) - math.log(n_phi)
            ml[i, sl] = np.max(lnl_ml(dh, hh), axis=1)
            dhs[i, sl], hhs[i, sl] = dh, hh
    lnp = np.asarray(ln_w_int)[:, None] + np.asarray(ln_w_ext)[None, :] + lnl
    return dict(lnl=lnl, ml_max=ml, dh=dhs, hh=hhs, lnp=lnp)


def evidence_general(res, n_norm, n_ext):
    """ln Z = LSE_ie ln p_ie - ln N_norm - ln N_ext (eq. Z_sum) from
    eval_pairs_general's output."""
    return float(_lse(res["lnp"].ravel())) - math.log(n_norm) - math.log(n_ext)


# --------------------------------------------------------------------------
# O14: extrinsic samples by importance sampling from arrival-time
# probabilities (Sec. IV E; App. C)
# --------------------------------------------------------------------------
def fibonacci_sky(n):
    """n sky points of equal area 4 pi / n (a Fibonacci lattice: z_s = 1 -
    (2 s + 1)/n, longitude s times the golden angle): lat, lon [n]."""
    s = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * s + 1.0) / n
    ga = math.pi * (3.0 - math.sqrt(5.0))
    lon = np.mod(s * ga, 2.0 * math.pi)
    return np.arcsin(z), lon


def arrival_time_series(h, modes, cos_iota, f, d, w, t0, dt, n_t, n_phi):
    """rho^2_{ck}(t_j) = 2 max_o lnL^ML_{ckoj} (eq. single_det_ML maximised
    over the phase: the distance-optimised SNR^2 of one detector with free
    polarisation amplitudes) on detector k's grid t0[k] + j dt, for the
    rows c of h: [C, K, n_t]."""
    out = np.empty((len(h), len(d), n_t))
    for c in range(len(h)):
        for k in range(len(d)):
            times = t0[k] + dt * np.arange(n_t)
            out[c, k] = 2.0 * np.max(single_detector_ml(h[c], modes, cos_iota[c], f, d[k], w[k],
                                                        times, n_phi), axis=0)
    return out


def proposal_table(rho2, t0, dt, det_r, sky_lat, sky_lon, tg_lo, tg_hi, n_tg, beta=0.5):
    """The proposal over cells (sky point s, geocentre-time cell j) of one
    intrinsic sample c: ln W_c(s, j) = sum_k ln p_ck(t_j - r_k . n_s / c)
    with t_j = tg_lo + (j + 1/2)(tg_hi - tg_lo)/n_tg, and the per-detector
    arrival-time probability p_ck(t) = exp(beta (rho^2_ck(t_i) - max_i
    rho^2_ck)) taken at the grid point t_i nearest to t (zero off the grid's
    cells).  Returns ln W [C, S, J] and ln Z_c = ln sum_sj W_c."""
    C, K, n_t = rho2.shape
    n = sky_direction(sky_lat, sky_lon)                                     # [S, 3]
    tau = -(n @ np.asarray(det_r).T) / C_SI                                 # [S, K]
    dtg = (tg_hi - tg_lo) / n_tg
    tj = tg_lo + (np.arange(n_tg) + 0.5) * dtg                              # [J]
    lnW = np.zeros((C, len(n), n_tg))
    for k in range(K):
        tk = tj[None, :] + tau[:, k:k + 1]                                  # [S, J]
        i = np.rint((tk - t0[k]) / dt).astype(np.int64)
        inside = (i >= 0) & (i < n_t)
        lp = beta * (rho2[:, k, :] - np.max(rho2[:, k, :], axis=1, keepdims=True))   # [C, n_t]
        term = np.where(inside[None], lp[:, np.clip(i, 0, n_t - 1)], -np.inf)
        lnW = lnW + term
    lnZ = np.array([_lse(lnW[c].ravel()) for c in range(C)])
    return lnW, lnZ


def extrinsic_proposal(lnW, lnZ, sky_lat, sky_lon, tg_lo, tg_hi, n_samples, seed):
    """Draws from the mixture of the C proposals (stratified: draw q from
    component q mod C): its cell by inverting the component's distribution
    over the cells (s-major) at u = SplitMix64(seed, 4 q), t_geo uniform in
    the cell's time at SplitMix64(seed, 4 q + 1), psi = pi u at 4 q + 2 and
    cos iota = 2 u - 1 at 4 q + 3 (prior); the importance weight of eq.
    (w_e): ln w = ln pi_cell - ln pi'_cell with the prior's cell probability
    1 / (S J) and the mixture's (1/C) sum_c W_c / Z_c.  Returns a dict of
    lat, lon, psi, cos_iota, t_geo, ln_w, cell [n_samples]."""
    C, S, J = lnW.shape
    P = np.exp(lnW - lnZ[:, None, None]).reshape(C, S * J)
    mix = np.log(np.mean(P, axis=0))                                        # ln pi'_cell
    dtg = (tg_hi - tg_lo) / J
    out = {k: np.empty(n_samples) for k in ("lat", "lon", "psi", "cos_iota", "t_geo", "ln_w")}
    out["cell"] = np.empty(n_samples, dtype=np.int64)
    for q in range(n_samples):
        c = q % C
        cell = inverse_cdf_index(P[c], splitmix64_uniform(seed, 4 * q))
        s, j = divmod(cell, J)
        out["cell"][q] = cell
        out["lat"][q], out["lon"][q] = sky_lat[s], sky_lon[s]
        out["t_geo"][q] = tg_lo + (j + splitmix64_uniform(seed, 4 * q + 1)) * dtg
        out["psi"][q] = math.pi * splitmix64_uniform(seed, 4 * q + 2)
        out["cos_iota"][q] = 2.0 * splitmix64_uniform(seed, 4 * q + 3) - 1.0
        out["ln_w"][q] = -math.log(S * J) - mix[cell]
    return out
