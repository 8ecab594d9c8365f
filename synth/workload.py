"""Seeded synthetic workloads for the likelihood-matrix hot path.

Test infrastructure and benchmark input only.  Nothing here evaluates the
likelihood: this module draws parameters, builds a synthetic waveform bank,
synthetic detectors, an analytic noise curve and simulated detector data.
Both the CPU oracle and the GPU library consume what it returns; neither
imports anything else from the other.

Stand-ins (the paper's own inputs -- IMRPhenomXODE banks, O3 noise curves,
GWTC-calibrated banks -- are not available):

* waveforms: inspiral-only TaylorF2 with 2PN point-particle phase and a
  1.5PN aligned-spin term, amplitude proportional to Mc^(5/6) f^(-7/6);
  higher modes follow Psi_lm(f) = (m/2) Psi_22(2f/m) with leading-order
  post-Newtonian amplitude ratios (configuration text of the workload);
* detectors: three synthetic L-shaped interferometers on a spherical Earth
  at fixed latitude, longitude and x-arm azimuth;
* noise: an analytic broadband fit of an advanced-LIGO-like curve,
  Gaussian noise drawn per frequency bin.

Units: frequencies in Hz, times in s, distances in Mpc, detector positions
in metres.  Waveforms are stored at the reference distance d0 (1 Mpc,
Sec. IV B) with reference phase 0 and polarisation angle 0 (Sec. IV A).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# physical constants (SI)
C_SI = 299792458.0
MPC_SI = 3.0856775814913673e22
GMSUN_S = 4.925490947641267e-06       # G M_sun / c^3 in seconds
EARTH_RADIUS_M = 6.371e6
MPC_S = MPC_SI / C_SI                 # 1 Mpc in light-seconds

# (l, m) channel sets used by the workloads
MODES_22 = ((2, 2),)
MODES_HM = ((2, 2), (2, 1), (3, 3), (3, 2), (4, 4))

# synthetic sites: latitude, longitude, x-arm azimuth (degrees; azimuth is
# measured from local East towards local North), relative noise amplitude
SITES = {
    "H": (46.5, -119.4, 126.0, 1.0),
    "L": (30.6, -90.8, 198.0, 1.0),
    "V": (43.6, 10.5, 70.6, 1.6),
}


# --------------------------------------------------------------------------
# detectors and noise
# --------------------------------------------------------------------------
@dataclass
class Network:
    names: tuple
    r: np.ndarray          # [K, 3] detector positions, metres, Earth-fixed
    D: np.ndarray          # [K, 3, 3] response tensors 0.5 (x x^T - y y^T)
    noise_amp: np.ndarray  # [K] multiplies the analytic noise amplitude


def network(names="HL") -> Network:
    rs, Ds, amps = [], [], []
    for n in names:
        lat, lon, az, amp = SITES[n]
        la, lo, a = np.radians(lat), np.radians(lon), np.radians(az)
        up = np.array([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)])
        east = np.array([-np.sin(lo), np.cos(lo), 0.0])
        north = np.cross(up, east)
        x = np.cos(a) * east + np.sin(a) * north
        y = np.cos(a + np.pi / 2) * east + np.sin(a + np.pi / 2) * north
        rs.append(EARTH_RADIUS_M * up)
        Ds.append(0.5 * (np.outer(x, x) - np.outer(y, y)))
        amps.append(amp)
    return Network(tuple(names), np.array(rs), np.array(Ds), np.array(amps))


def psd(f, amp=1.0):
    """One-sided analytic noise PSD [1/Hz] (broadband aLIGO-like fit)."""
    x = np.asarray(f, dtype=np.float64) / 215.0
    s = x ** -4.14 - 5.0 / x ** 2 + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2)
    return 1e-49 * s * amp ** 2


def freq_bins(n_bins, f_lo=20.0, f_hi=512.0):
    return f_lo * (f_hi / f_lo) ** (np.arange(n_bins) / (n_bins - 1.0))


def bin_widths(f):
    """Trapezoid widths for a non-uniform grid (half intervals at the ends)."""
    f = np.asarray(f, dtype=np.float64)
    df = np.empty_like(f)
    df[1:-1] = 0.5 * (f[2:] - f[:-2])
    df[0] = 0.5 * (f[1] - f[0])
    df[-1] = 0.5 * (f[-1] - f[-2])
    return df


def psd_weights(f, net: Network):
    """w_kb = 4 df_b / S_k(f_b): the per-bin weights of the noise-weighted
    inner product (Sec. III A, summed over the bins)."""
    df = bin_widths(f)
    return np.stack([4.0 * df / psd(f, a) for a in net.noise_amp])


# --------------------------------------------------------------------------
# waveform bank
# --------------------------------------------------------------------------
def draw_intrinsic(rng, n, mc_range, q_range, chi_range=(0.0, 0.0)):
    """Chirp mass log-uniform, mass ratio (<=1) uniform, chi_eff uniform."""
    lo, hi = np.log(mc_range[0]), np.log(mc_range[1])
    mc = np.exp(rng.uniform(lo, hi, n))
    q = rng.uniform(q_range[0], q_range[1], n)
    chi = rng.uniform(chi_range[0], chi_range[1], n) if chi_range[1] > chi_range[0] \
        else np.full(n, float(chi_range[0]))
    return mc, q, chi


def _amp_ratio(l, m, v, delta, eta, xp):
    if (l, m) == (2, 2):
        return xp.ones_like(v)
    if (l, m) == (2, 1):
        return (math.sqrt(2.0) / 3.0) * delta * v
    if (l, m) == (3, 3):
        return 0.75 * math.sqrt(15.0 / 14.0) * delta * v
    if (l, m) == (3, 2):
        return (1.0 / 3.0) * math.sqrt(5.0 / 7.0) * (1.0 - 3.0 * eta) * v * v
    if (l, m) == (4, 4):
        return (4.0 / 9.0) * math.sqrt(10.0 / 7.0) * (1.0 - 3.0 * eta) * v * v
    raise ValueError(f"no amplitude model for mode {(l, m)}")


def waveform_modes(f, mc, q, chi, modes, xp=np, d0_mpc=1.0):
    """Frequency-domain mode amplitudes h_c(f_b) at distance d0, phi=0, psi=0.

    f: [N_b]; mc, q, chi: [N] arrays (either numpy, or torch tensors with
    xp=torch, float64).  Returns complex [N, N_c, N_b].
    """
    f = xp.asarray(f) if xp is np else f
    mc = mc[:, None]
    q = q[:, None]
    chi = chi[:, None]
    eta = q / (1.0 + q) ** 2
    delta = (1.0 - q) / (1.0 + q)
    mtot_s = mc * GMSUN_S / eta ** 0.6
    mc_s = mc * GMSUN_S
    d_s = d0_mpc * MPC_S
    f_isco22 = 1.0 / (6.0 ** 1.5 * math.pi * mtot_s)
    beta = (113.0 / 12.0 - 19.0 / 3.0 * eta) * chi
    a2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta
    a3 = -16.0 * math.pi + 4.0 * beta
    a4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * eta ** 2
    out = []
    for (l, m) in modes:
        F = 2.0 * f[None, :] / m                    # equivalent 22 frequency
        v = (math.pi * mtot_s * F) ** (1.0 / 3.0)
        psi22 = -math.pi / 4 + 3.0 / (128.0 * eta * v ** 5) * (
            1.0 + a2 * v ** 2 + a3 * v ** 3 + a4 * v ** 4)
        phase = 0.5 * m * psi22
        amp = math.sqrt(2.0 * math.pi / 3.0) * math.pi ** (-2.0 / 3.0) \
            * mc_s ** (5.0 / 6.0) * F ** (-7.0 / 6.0) / d_s
        amp = amp * _amp_ratio(l, m, v, delta, eta, xp)
        amp = xp.where(F < f_isco22, amp, xp.zeros_like(amp))
        out.append(amp * (xp.cos(phase) - 1j * xp.sin(phase)))
    return xp.stack(out, axis=1)


def bank_on_device(torch, mc, q, chi, f, modes, chunk=32768):
    """The bank of waveform_modes built on the GPU with torch in float64, as a
    [N, N_c, N_b, 2] tensor (interleaved complex), chunk by chunk: banks of
    the large workloads are generated where they are used."""
    n = len(mc)
    out = torch.empty((n, len(modes), len(f), 2), dtype=torch.float64, device="cuda")
    ft = torch.as_tensor(np.asarray(f), dtype=torch.float64, device="cuda")
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        args = [torch.as_tensor(np.asarray(x[s:e]), dtype=torch.float64, device="cuda")
                for x in (mc, q, chi)]
        out[s:e] = torch.view_as_real(waveform_modes(ft, *args, modes, xp=torch))
    torch.cuda.synchronize()
    return out


# --------------------------------------------------------------------------
# extrinsic samples
# --------------------------------------------------------------------------
def draw_extrinsic(rng, n, t_window=0.01):
    """Prior draws: isotropic sky (Earth-fixed latitude/longitude), uniform
    polarisation angle, uniform cos(inclination), uniform geocentre time."""
    return dict(
        lat=np.arcsin(rng.uniform(-1.0, 1.0, n)),
        lon=rng.uniform(0.0, 2 * np.pi, n),
        psi=rng.uniform(0.0, np.pi, n),
        cos_iota=rng.uniform(-1.0, 1.0, n),
        t_geo=rng.uniform(-t_window, t_window, n),
    )


# --------------------------------------------------------------------------
# forward simulation of detector data (injections)
# --------------------------------------------------------------------------
def _swsh_m2(l, m, cos_t):
    """Spin-weight -2 spherical harmonic at azimuth 0 (Goldberg's sum)."""
    s = -2
    th = np.arccos(np.clip(cos_t, -1.0, 1.0))
    pref = (-1.0) ** m * math.sqrt(
        math.factorial(l + m) * math.factorial(l - m) * (2 * l + 1)
        / (4 * math.pi * math.factorial(l + s) * math.factorial(l - s)))
    half = th / 2.0
    tot = 0.0
    for r in range(0, l - s + 1):
        k = r + s - m
        if k < 0 or k > l + s:
            continue
        c = math.comb(l - s, r) * math.comb(l + s, k) * (-1.0) ** (l - r - s)
        # sin^(2l)(t/2) cot^(2r+s-m)(t/2) written without dividing by sin
        p = 2 * r + s - m
        tot = tot + c * np.cos(half) ** p * np.sin(half) ** (2 * l - p)
    return pref * tot


def simulate_strain(h_modes, modes, f, net: Network, ext_one: dict, phi_ref, dist_mpc,
                    d0_mpc=1.0):
    """Detector strain of one source: [K, N_b] complex.

    h_modes [N_c, N_b] at d0; ext_one holds scalar lat, lon, psi, cos_iota,
    t_geo.  Source direction n (towards the source), polarisation basis
    X = cos(psi) e_lon + sin(psi) e_lat, Y = -sin(psi) e_lon + cos(psi) e_lat,
    e_+ = XX^T - YY^T, e_x = XY^T + YX^T, detector time t_geo - r.n/c,
    orbital phase factor exp(-i m phi_ref), amplitude d0/D.
    """
    la, lo, ps = ext_one["lat"], ext_one["lon"], ext_one["psi"]
    n = np.array([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)])
    e_lon = np.array([-np.sin(lo), np.cos(lo), 0.0])
    e_lat = np.array([-np.sin(la) * np.cos(lo), -np.sin(la) * np.sin(lo), np.cos(la)])
    X = np.cos(ps) * e_lon + np.sin(ps) * e_lat
    Y = -np.sin(ps) * e_lon + np.cos(ps) * e_lat
    ep = np.outer(X, X) - np.outer(Y, Y)
    ex = np.outer(X, Y) + np.outer(Y, X)
    out = np.zeros((len(net.names), len(f)), dtype=np.complex128)
    ci = ext_one["cos_iota"]
    for k in range(len(net.names)):
        fp = float(np.sum(net.D[k] * ep))
        fx = float(np.sum(net.D[k] * ex))
        tk = ext_one["t_geo"] - float(net.r[k] @ n) / C_SI
        for c, (l, m) in enumerate(modes):
            ylm_neg = _swsh_m2(l, -m, ci)
            ylm_pos = _swsh_m2(l, m, ci)
            kp = 0.5 * (ylm_neg + (-1) ** l * ylm_pos)
            kx = 0.5j * (ylm_neg - (-1) ** l * ylm_pos)
            out[k] += h_modes[c] * (fp * kp + fx * kx) * np.exp(-1j * m * phi_ref)
        out[k] *= np.exp(-2j * np.pi * f * tk)
    return out * (d0_mpc / dist_mpc)


def noise(rng, w):
    """Gaussian noise per bin: n = (x + i y)/sqrt(w), so Re<n|h> ~ N(0, <h|h>)."""
    x = rng.standard_normal(w.shape)
    y = rng.standard_normal(w.shape)
    return (x + 1j * y) / np.sqrt(w)


def optimal_snr2(strain, w):
    return float(np.sum(w * np.abs(strain) ** 2))


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    """Everything both paths take as input (host arrays, float64)."""
    modes: tuple
    f: np.ndarray                  # [N_b]
    h: np.ndarray                  # [N_i, N_c, N_b] complex
    ln_w_int: np.ndarray           # [N_i]
    det_r: np.ndarray              # [K, 3]
    det_D: np.ndarray              # [K, 3, 3]
    d: np.ndarray                  # [K, N_b] complex
    w: np.ndarray                  # [K, N_b]
    ext: dict                      # lat, lon, psi, cos_iota, t_geo [N_e]
    ln_w_ext: np.ndarray           # [N_e]
    n_phi: int
    d_max: float = 5000.0
    d0: float = 1.0
    n_norm: float = 0.0            # 0 -> number of bank rows used
    meta: dict = field(default_factory=dict)

    @property
    def n_int(self):
        return self.h.shape[0]

    @property
    def n_ext(self):
        return len(self.ln_w_ext)

    @property
    def mode_l(self):
        return np.array([l for l, _ in self.modes], dtype=np.int32)

    @property
    def mode_m(self):
        return np.array([m for _, m in self.modes], dtype=np.int32)

    def subset(self, rows=None, cols=None):
        """A smaller workload on a subset of bank rows / extrinsic samples."""
        rows = np.arange(self.n_int) if rows is None else np.asarray(rows)
        cols = np.arange(self.n_ext) if cols is None else np.asarray(cols)
        return Workload(self.modes, self.f, self.h[rows], self.ln_w_int[rows], self.det_r,
                        self.det_D, self.d, self.w, {k: v[cols] for k, v in self.ext.items()},
                        self.ln_w_ext[cols], self.n_phi, self.d_max, self.d0, self.n_norm,
                        dict(self.meta))


def make_workload(seed, n_int, n_ext, n_bins, modes, dets, n_phi, snr,
                  mc_range, q_range, chi_range=(0.0, 0.0), noise_on=True,
                  in_bank=False, random_weights=False, d_max=5000.0, d0=1.0,
                  f_lo=20.0, f_hi=512.0, with_bank=True):
    """Build one synthetic event against a synthetic bank.

    snr: optimal network SNR of the injected source (its distance is set to
    reach it).  in_bank=True injects bank member 0 at extrinsic sample 0 and
    grid phase index n_phi//4 without noise unless noise_on (a
    zero-noise in-bank injection has lnL = rho^2/2 at that triple).
    """
    rng = np.random.default_rng(seed)
    net = network(dets)
    f = freq_bins(n_bins, f_lo, f_hi)
    w = psd_weights(f, net)
    mc, q, chi = draw_intrinsic(rng, n_int, mc_range, q_range, chi_range)
    h = waveform_modes(f, mc, q, chi, modes) if with_bank else None
    ext = draw_extrinsic(rng, n_ext)
    if random_weights:
        ln_w_int = rng.normal(0.0, 0.5, n_int)
        ln_w_ext = rng.normal(0.0, 0.5, n_ext)
    else:
        ln_w_int = np.zeros(n_int)
        ln_w_ext = np.zeros(n_ext)
    meta = dict(seed=seed, mc=mc, q=q, chi=chi, snr=snr, dets=dets)
    if in_bank:
        hi = h[0] if with_bank else waveform_modes(f, mc[:1], q[:1], chi[:1], modes)[0]
        ext1 = {k: v[0] for k, v in ext.items()}
        o_star = n_phi // 4
        phi = 2 * np.pi * o_star / n_phi
        s0 = simulate_strain(hi, modes, f, net, ext1, phi, d0, d0)
        dist = d0 * math.sqrt(optimal_snr2(s0, w)) / snr
        meta.update(inj_i=0, inj_e=0, inj_o=o_star, inj_dist=dist)
    else:
        mci, qi, chii = draw_intrinsic(rng, 1, mc_range, q_range, chi_range)
        # keep the injected source away from the bank edge
        hi = waveform_modes(f, mci, qi, chii, modes)[0]
        ext1 = {k: v[0] for k, v in draw_extrinsic(rng, 1).items()}
        phi = rng.uniform(0, 2 * np.pi)
        s0 = simulate_strain(hi, modes, f, net, ext1, phi, d0, d0)
        dist = d0 * math.sqrt(optimal_snr2(s0, w)) / snr
        meta.update(inj_mc=float(mci[0]), inj_q=float(qi[0]), inj_chi=float(chii[0]),
                    inj_ext=ext1, inj_phi=phi, inj_dist=dist)
    d = s0 * (d0 / dist)
    if noise_on:
        d = d + noise(rng, w)
    return Workload(tuple(modes), f, h, ln_w_int, net.r.copy(), net.D.copy(), d, w, ext,
                    ln_w_ext, n_phi, d_max, d0, 0.0, meta)


# Named configurations (sizes and distributions of the workloads)
def config_tiny(seed=0, snr=15.0, **kw):
    """2 detectors, 22 only, 64 log bins in 20-512 Hz, 256 x 512, 16 phases."""
    args = dict(n_int=256, n_ext=512, n_bins=64, modes=MODES_22, dets="HL", n_phi=16,
                snr=snr, mc_range=(10.0, 40.0), q_range=(0.2, 1.0))
    args.update(kw)
    return make_workload(seed, **args)


def config_production(seed=1, snr=20.0, n_int=65536, n_ext=4096, **kw):
    """3 detectors, 5 modes, 256 bins, 65536 x 4096, 32 phases."""
    args = dict(n_int=n_int, n_ext=n_ext, n_bins=256, modes=MODES_HM, dets="HLV", n_phi=32,
                snr=snr, mc_range=(5.0, 80.0), q_range=(0.1, 1.0), chi_range=(-0.9, 0.9))
    args.update(kw)
    return make_workload(seed, **args)


def config_large(seed=3, snr=20.0, n_int=1 << 20, n_ext=16384, **kw):
    """Large-bank streaming shape: 2^20 x 16384, 3 det, 5 modes, 256 bins."""
    return config_production(seed=seed, snr=snr, n_int=n_int, n_ext=n_ext, **kw)


# --------------------------------------------------------------------------
# the paper's own layout, (m, p) channels with the inclination in the bank
# (Sec. IV A), and full-resolution events for relative binning (App. A)
# --------------------------------------------------------------------------
def mp_channels(modes):
    """The (m, p) channels of the distinct m of `modes`: m ascending, + (0) then x (1)."""
    ms = sorted({m for _, m in modes})
    return tuple((m, p) for m in ms for p in (0, 1))


def waveform_mp(f, mc, q, chi, cos_iota, modes):
    """h_{mp}(f) [N, 2 N_m, N_b] at d0, phi = 0, psi = 0 for rows with
    inclination cos_iota [N]: the + and x polarisations of each azimuthal
    harmonic m, i.e. the (l, m) modes of waveform_modes summed over l with
    the polarisation factors simulate_strain uses."""
    hlm = waveform_modes(f, mc, q, chi, modes)
    chans = mp_channels(modes)
    ci = np.asarray(cos_iota, dtype=np.float64)
    out = np.zeros((hlm.shape[0], len(chans), hlm.shape[2]), dtype=np.complex128)
    for c, (l, m) in enumerate(modes):
        yn = _swsh_m2(l, -m, ci)
        yp = _swsh_m2(l, m, ci)
        j = chans.index((m, 0))
        out[:, j] += (0.5 * (yn + (-1) ** l * yp))[:, None] * hlm[:, c]
        out[:, j + 1] += (0.5j * (yn - (-1) ** l * yp))[:, None] * hlm[:, c]
    return out, chans


@dataclass
class RBEvent:
    """A full-resolution event for relative binning, and a bank on its nodes."""
    f_full: np.ndarray             # [F] Hz, uniform grid
    d_full: np.ndarray             # [K, F] complex
    w_full: np.ndarray             # [K, F] 4 df / S_k(f)
    node_idx: np.ndarray           # [B] indices of the spline nodes in f_full
    h0: np.ndarray                 # [C, F] reference channels (the bank's layout)
    t0: np.ndarray                 # [K] reference arrival time per detector, s
    layout: str                    # "lm": (l, m) channels; "mp": (m, p) channels
    chans: tuple                   # (l, m) or (m, p) per channel
    wl: Workload                   # bank on the nodes, detectors, extrinsic set


def make_rb_event(seed, n_int, n_ext, n_bins, n_full, modes=MODES_HM, dets="HLV", n_phi=32,
                  snr=20.0, layout="lm", mc0=4.0, q0=0.6, spread=0.01, f_lo=20.0, f_hi=200.0,
                  t_spread=5e-4, noise_on=True):
    """An injection at (mc0, q0, chi 0) observed on a uniform full-resolution
    grid with noise; the reference waveform is the injection's own channels
    with its detector arrival times; the bank (rows within `spread` of mc0
    in chirp mass, q0 +- 0.05) is evaluated on n_bins log-spaced nodes of the
    grid; the extrinsic samples put the source within t_spread of the
    injection's arrival time (sky and inclination drawn as usual)."""
    rng = np.random.default_rng(seed)
    net = network(dets)
    f_full = np.linspace(f_lo, f_hi, n_full)
    w_full = psd_weights(f_full, net)
    want = f_lo * (f_hi / f_lo) ** (np.arange(n_bins) / (n_bins - 1.0))
    node_idx = np.unique(np.clip(np.round((want - f_lo) / (f_full[1] - f_full[0])), 0, n_full - 1)
                         .astype(np.int64))
    f_nodes = f_full[node_idx]
    mc = mc0 * np.exp(rng.uniform(-spread, spread, n_int))
    q = np.clip(q0 + rng.uniform(-0.05, 0.05, n_int), 0.1, 1.0)
    chi = np.zeros(n_int)
    ext1 = {k: v[0] for k, v in draw_extrinsic(rng, 1).items()}
    phi = rng.uniform(0, 2 * np.pi)
    h_inj = waveform_modes(f_full, np.array([mc0]), np.array([q0]), np.array([0.0]), modes)[0]
    s0 = simulate_strain(h_inj, modes, f_full, net, ext1, phi, 1.0, 1.0)
    dist = math.sqrt(optimal_snr2(s0, w_full)) / snr
    d_full = s0 / dist
    if noise_on:
        d_full = d_full + noise(rng, w_full)
    n = np.array([np.cos(ext1["lat"]) * np.cos(ext1["lon"]), np.cos(ext1["lat"]) * np.sin(ext1["lon"]),
                  np.sin(ext1["lat"])])
    t0 = ext1["t_geo"] - net.r @ n / C_SI
    if layout == "lm":
        h = waveform_modes(f_nodes, mc, q, chi, modes)
        h0 = h_inj
        chans = tuple(modes)
    else:
        h, chans = waveform_mp(f_nodes, mc, q, chi, rng.uniform(-0.9, 0.9, n_int), modes)
        h0 = waveform_mp(f_full, np.array([mc0]), np.array([q0]), np.array([0.0]),
                         np.array([ext1["cos_iota"]]), modes)[0][0]
    ext = draw_extrinsic(rng, n_ext)
    ext["lat"] = ext1["lat"] + rng.normal(0.0, 0.02, n_ext)
    ext["lon"] = ext1["lon"] + rng.normal(0.0, 0.02, n_ext)
    ext["t_geo"] = ext1["t_geo"] + rng.uniform(-t_spread, t_spread, n_ext)
    wl = Workload(tuple(chans), f_nodes, h, np.zeros(n_int), net.r.copy(), net.D.copy(),
                  d_full[:, node_idx], w_full[:, node_idx], ext, np.zeros(n_ext), n_phi,
                  meta=dict(seed=seed, mc=mc, q=q, chi=chi, snr=snr, dets=dets, inj_ext=ext1,
                            inj_phi=phi, inj_dist=dist, layout=layout))
    return RBEvent(f_full, d_full, w_full, node_idx, h0, t0, layout, tuple(chans), wl)
