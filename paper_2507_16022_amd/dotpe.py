"""Python binding of the C ABI in include/dotpe.h (argument marshalling only).

Every computation runs in libdotpe.so's HIP kernels.  numpy arrays are
passed as host pointers; torch tensors on a GPU are passed as device
pointers (torch is used only for device memory and streams).  If the
library has not been built this module raises on first use: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdotpe.so")

OK = 0
E_INVALID_ARG = -1
E_OOM = -2
E_ADMISSION = -3
E_NUMERIC = -4
E_DEVICE = -5
E_TOO_LARGE = -6
E_UNIMPLEMENTED = -7

PREC = {"fp64": 0, "fp16x2": 1, "bf16x2": 2}
MEM_HOST, MEM_DEVICE = 0, 1

_c_dp = ctypes.POINTER(ctypes.c_double)
_c_ip = ctypes.POINTER(ctypes.c_int32)
_c_lp = ctypes.POINTER(ctypes.c_int64)


class BankDesc(ctypes.Structure):
    _fields_ = [("n_wf", ctypes.c_int64), ("n_modes", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("mode_l", ctypes.c_void_p), ("mode_m", ctypes.c_void_p),
                ("f_bins", ctypes.c_void_p), ("h", ctypes.c_void_p), ("ln_w", ctypes.c_void_p),
                ("precision", ctypes.c_int32), ("mem", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("mode_p", ctypes.c_void_p)]


LAYOUT = {"lm": 0, "mp": 1}


class EventDesc(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("d", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("det_r", ctypes.c_void_p), ("det_D", ctypes.c_void_p),
                ("n_ext", ctypes.c_int64),
                ("lat", ctypes.c_void_p), ("lon", ctypes.c_void_p), ("psi", ctypes.c_void_p),
                ("cos_iota", ctypes.c_void_p), ("t_geo", ctypes.c_void_p),
                ("ln_w_ext", ctypes.c_void_p),
                ("d_max", ctypes.c_double), ("d0", ctypes.c_double), ("n_norm", ctypes.c_double),
                ("sub_start", ctypes.c_int64), ("sub_count", ctypes.c_int64),
                ("sub_idx", ctypes.c_void_p),
                ("cut_delta", ctypes.c_double), ("top_k", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("topk_window", ctypes.c_double),
                ("stream", ctypes.c_void_p), ("cut_target", ctypes.c_double),
                ("w_dh", ctypes.c_void_p), ("w_hh", ctypes.c_void_p), ("dd", ctypes.c_double)]


class ExtrinsicDesc(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("n_t", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("n_rows", ctypes.c_int32), ("d", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("det_r", ctypes.c_void_p), ("t0", ctypes.c_void_p), ("dt", ctypes.c_double),
                ("rows", ctypes.c_void_p), ("cos_iota", ctypes.c_void_p), ("beta", ctypes.c_double),
                ("n_sky", ctypes.c_int32), ("n_tg", ctypes.c_int32), ("tg_lo", ctypes.c_double),
                ("tg_hi", ctypes.c_double), ("n_samples", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_void_p)]


class ExtrinsicResult(ctypes.Structure):
    _fields_ = [("n_eff_prior", ctypes.c_double), ("support", ctypes.c_double),
                ("t_ms", ctypes.c_double), ("n_samples", ctypes.c_int64)]


class RBDesc(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("n_modes", ctypes.c_int32), ("n_full", ctypes.c_int64),
                ("f", ctypes.c_void_p), ("d", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("h0", ctypes.c_void_p), ("t0", ctypes.c_void_p), ("n_nodes", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("node_idx", ctypes.c_void_p)]


class EvidenceResult(ctypes.Structure):
    _fields_ = [("ln_z", ctypes.c_double), ("ln_z_upper", ctypes.c_double),
                ("max_lnl_ml", ctypes.c_double), ("ln_sum_p", ctypes.c_double),
                ("ln_sum_p2", ctypes.c_double), ("dd", ctypes.c_double),
                ("max_ln_p", ctypes.c_double),
                ("n_pairs", ctypes.c_int64), ("n_pairs_bounded", ctypes.c_int64),
                ("n_triples_marg", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("topk_count", ctypes.c_int32), ("topk_exact", ctypes.c_int32),
                ("status", ctypes.c_int32), ("t_pilot_ms", ctypes.c_double),
                ("t_fused_ms", ctypes.c_double), ("cut_delta_used", ctypes.c_double),
                ("n_passes", ctypes.c_int32), ("n_tiles_rerun", ctypes.c_int32),
                ("t_main_ms", ctypes.c_double), ("n_tiles_listed", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("ln_sum_p2_triples", ctypes.c_double),
                ("ln_sum_row2", ctypes.c_double), ("ln_sum_col2", ctypes.c_double)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("pool_bytes", ctypes.c_uint64), ("batch_pairs", ctypes.c_uint64)]


class TicketInfo(ctypes.Structure):
    _fields_ = [("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("bytes", ctypes.c_uint64),
                ("slot", ctypes.c_int32), ("status", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PreselectDesc(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int32), ("n_t", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("d", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("t0", ctypes.c_void_p), ("dt", ctypes.c_double), ("cos_iota", ctypes.c_void_p),
                ("sub_start", ctypes.c_int64), ("sub_count", ctypes.c_int64),
                ("delta_lnl", ctypes.c_double), ("stream", ctypes.c_void_p)]


class PreselectResult(ctypes.Structure):
    _fields_ = [("lnl_max", ctypes.c_double), ("threshold", ctypes.c_double),
                ("n_rows", ctypes.c_int64), ("n_selected", ctypes.c_int64), ("t_ms", ctypes.c_double)]


class PosteriorSample(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int64), ("e", ctypes.c_int64), ("o", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("distance", ctypes.c_double),
                ("ln_p_pair", ctypes.c_double), ("ln_p_triple", ctypes.c_double)]


class Sample(ctypes.Structure):
    _fields_ = [("i", ctypes.c_int64), ("e", ctypes.c_int64), ("ln_p", ctypes.c_double),
                ("o_best", ctypes.c_int32), ("reserved", ctypes.c_int32)]


SYMBOLS = {
    "dotpe_version": (ctypes.c_char_p, []),
    "dotpe_last_error": (ctypes.c_char_p, []),
    "dotpe_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]),
    "dotpe_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "dotpe_device_bytes": (ctypes.c_uint64, [ctypes.c_void_p]),
    "dotpe_load_bank": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BankDesc),
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "dotpe_free_bank": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "dotpe_set_event": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(EventDesc),
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "dotpe_free_event": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "dotpe_eval_lnl": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "dotpe_evidence": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.POINTER(EvidenceResult), ctypes.c_void_p]),
    "dotpe_evidence_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(EventDesc),
                                              ctypes.POINTER(EvidenceResult), ctypes.c_void_p]),
    "dotpe_event_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(EventDesc),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "dotpe_sample_posterior": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                               ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p,
                                               ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "dotpe_preselect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(PreselectDesc),
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(PreselectResult)]),
    "dotpe_rb_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RBDesc), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "dotpe_extrinsic_samples": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.POINTER(ExtrinsicDesc)] + [ctypes.c_void_p] * 6
                                + [ctypes.POINTER(ExtrinsicResult)]),
    "dotpe_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ServerDesc),
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "dotpe_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "dotpe_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(EventDesc),
                                     ctypes.POINTER(ctypes.c_int64)]),
    "dotpe_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]),
    "dotpe_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(EvidenceResult),
                                   ctypes.c_void_p, ctypes.POINTER(TicketInfo)]),
}

# include/dotpe_test.h: hooks the parity tests use to check single steps
TEST_SYMBOLS = {
    "dotpe_debug_distmarg": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]),
    "dotpe_debug_response": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "dotpe_debug_bound": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libdotpe.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with __graft_entry__.build() "
                           "(python paper_2507_16022_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in list(SYMBOLS.items()) + list(TEST_SYMBOLS.items()):
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DotpeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dotpe error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise DotpeError(rc, load_library().dotpe_last_error().decode())


def _host(a, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class Context:
    def __init__(self, device=0, budget_bytes=0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.dotpe_create(int(device), int(budget_bytes), ctypes.byref(h)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def device_bytes(self):
        return int(load_library().dotpe_device_bytes(self._h))

    def close(self):
        if self._h:
            load_library().dotpe_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_bank(self, h, modes, f, ln_w=None, precision="fp16x2", layout="lm"):
        """h: complex numpy [N, C, B] (host) or a float64 torch tensor
        [N, C, B, 2] on the GPU (device pointer, no host copy).  modes: (l, m) per
        channel (layout "lm") or (m, p) per channel (layout "mp", p 0 for +, 1 for x)."""
        return Bank(self, h, modes, f, ln_w, precision, layout)

    def extrinsic_samples(self, bank, d, w, det_r, t0, dt, n_t, rows, cos_iota, n_phi, n_sky, n_tg,
                          tg_lo, tg_hi, n_samples, seed=0, beta=0.5, stream=None):
        """dotpe_extrinsic_samples: importance-sampled extrinsic parameters from the
        arrival-time probabilities of the intrinsic samples `rows`.  Returns a dict with
        lat, lon, psi, cos_iota, t_geo, ln_w [n_samples] and the result fields."""
        d = np.ascontiguousarray(d, dtype=np.complex128)
        w = np.ascontiguousarray(w, dtype=np.float64)
        r = np.ascontiguousarray(det_r, dtype=np.float64)
        t0 = np.ascontiguousarray(t0, dtype=np.float64)
        rw = np.ascontiguousarray(rows, dtype=np.int64)
        ci = np.ascontiguousarray(cos_iota, dtype=np.float64)
        if stream is not None and not isinstance(stream, int):
            stream = stream.cuda_stream
        desc = ExtrinsicDesc(d.shape[0], int(n_t), int(n_phi), len(rw), d.ctypes.data, w.ctypes.data,
                             r.ctypes.data, t0.ctypes.data, float(dt), rw.ctypes.data, ci.ctypes.data,
                             float(beta), int(n_sky), int(n_tg), float(tg_lo), float(tg_hi),
                             int(n_samples), ctypes.c_uint64(int(seed)), stream)
        out = {k: np.empty(int(n_samples)) for k in ("lat", "lon", "psi", "cos_iota", "t_geo", "ln_w")}
        res = ExtrinsicResult()
        _check(load_library().dotpe_extrinsic_samples(
            self._h, bank.handle, ctypes.byref(desc), out["lat"].ctypes.data, out["lon"].ctypes.data,
            out["psi"].ctypes.data, out["cos_iota"].ctypes.data, out["t_geo"].ctypes.data,
            out["ln_w"].ctypes.data, ctypes.byref(res)))
        out.update({name: getattr(res, name) for name, _ in ExtrinsicResult._fields_})
        return out

    def rb_weights(self, f, d, w, h0, node_idx, t0=None):
        """dotpe_rb_weights: relative-binning weights from full-resolution data f [F],
        d [K, F] complex, w [K, F], reference channels h0 [C, F] complex, spline nodes
        node_idx [B] and reference arrival times t0 [K].  Returns (w_dh [K, C, B],
        w_hh [K, C, C, B], dd)."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.complex128)
        w = np.ascontiguousarray(w, dtype=np.float64)
        h0 = np.ascontiguousarray(h0, dtype=np.complex128)
        idx = np.ascontiguousarray(node_idx, dtype=np.int64)
        t0a = None if t0 is None else np.ascontiguousarray(t0, dtype=np.float64)
        K, C, B = d.shape[0], h0.shape[0], len(idx)
        desc = RBDesc(K, C, len(f), f.ctypes.data, d.ctypes.data, w.ctypes.data, h0.ctypes.data,
                      None if t0a is None else t0a.ctypes.data, B, 0, idx.ctypes.data)
        wdh = np.empty((K, C, B), dtype=np.complex128)
        whh = np.empty((K, C, C, B), dtype=np.complex128)
        dd = ctypes.c_double()
        _check(load_library().dotpe_rb_weights(self._h, ctypes.byref(desc), wdh.ctypes.data,
                                                whh.ctypes.data, ctypes.byref(dd)))
        return wdh, whh, dd.value

    def set_event(self, bank, **kw):
        return Event(self, bank, **kw)

    def evidence_static(self, bank, **kw):
        """dotpe_evidence_static: stage and evaluate one event in the library's fixed device
        scratch, allocating no device memory (same keywords as set_event)."""
        desc, keep = _event_desc(**kw)
        r = EvidenceResult()
        k = desc.top_k
        arr = (Sample * max(k, 1))()
        _check(load_library().dotpe_evidence_static(
            self._h, bank.handle, ctypes.byref(desc), ctypes.byref(r),
            ctypes.cast(arr, ctypes.c_void_p) if k else None))
        return _result(r, arr)

    def preselect(self, bank, d, w, t0, dt, n_t, cos_iota, n_phi, sub_start=0, sub_count=0,
                  delta_lnl=20.0, stream=None):
        """dotpe_preselect: each row's incoherent maximum likelihood over the (phase, time)
        grid and the rows within delta_lnl of the best.  Returns a dict with lnl_inco
        [rows], lnl_det [rows, n_det], selected (absolute bank rows, ascending) and the
        result fields."""
        d = np.ascontiguousarray(d, dtype=np.complex128)
        w = np.ascontiguousarray(w, dtype=np.float64)
        t0 = np.ascontiguousarray(t0, dtype=np.float64)
        ci = np.ascontiguousarray(cos_iota, dtype=np.float64)
        n_rows = len(ci)
        if sub_count == 0:
            sub_count = n_rows
        if stream is not None and not isinstance(stream, int):
            stream = stream.cuda_stream
        desc = PreselectDesc(d.shape[0], int(n_t), int(n_phi), 0, d.ctypes.data, w.ctypes.data,
                             t0.ctypes.data, float(dt), ci.ctypes.data, int(sub_start),
                             int(sub_count), float(delta_lnl), stream)
        lnl = np.empty(n_rows)
        per = np.empty((n_rows, d.shape[0]))
        sel = np.empty(n_rows, dtype=np.int64)
        r = PreselectResult()
        _check(load_library().dotpe_preselect(self._h, bank.handle, ctypes.byref(desc),
                                              lnl.ctypes.data, per.ctypes.data, sel.ctypes.data,
                                              ctypes.byref(r)))
        out = {name: getattr(r, name) for name, _ in PreselectResult._fields_}
        out.update(lnl_inco=lnl, lnl_det=per, selected=sel[:r.n_selected].copy())
        return out

    def distmarg(self, dh, hh, r0):
        dh, pdh = _host(dh)
        hh, phh = _host(hh)
        out = np.empty_like(dh)
        _check(load_library().dotpe_debug_distmarg(self._h, dh.size, pdh, phh, float(r0),
                                                   out.ctypes.data))
        return out


class Bank:
    def __init__(self, ctx, h, modes, f, ln_w=None, precision="fp16x2", layout="lm"):
        lib = load_library()
        self.ctx = ctx
        self._keep = []
        if layout == "mp":          # channels (m, p)
            ml, pml = _host([0 for _ in modes], np.int32)
            mm, pmm = _host([m for m, _ in modes], np.int32)
            mp_, pmp = _host([p for _, p in modes], np.int32)
        else:                       # channels (l, m)
            ml, pml = _host([l for l, _ in modes], np.int32)
            mm, pmm = _host([m for _, m in modes], np.int32)
            mp_, pmp = None, None
        fb, pf = _host(f)
        self._keep += [ml, mm, fb, mp_]
        if _is_torch(h):
            assert h.is_cuda and str(h.dtype) == "torch.float64" and h.is_contiguous()
            n_wf, n_c, n_b = h.shape[0], h.shape[1], h.shape[2]
            ph, mem = h.data_ptr(), MEM_DEVICE
            self._keep.append(h)
            if ln_w is not None:
                assert _is_torch(ln_w) and ln_w.is_cuda
                pw = ln_w.data_ptr()
                self._keep.append(ln_w)
            else:
                pw = None
        else:
            hh = np.ascontiguousarray(h, dtype=np.complex128)
            n_wf, n_c, n_b = hh.shape
            ph, mem = hh.ctypes.data, MEM_HOST
            self._keep.append(hh)
            if ln_w is not None:
                lw, pw = _host(ln_w)
                self._keep.append(lw)
            else:
                pw = None
        desc = BankDesc(n_wf, n_c, n_b, pml, pmm, pf, ph, pw, PREC[precision], mem, LAYOUT[layout], 0,
                        pmp)
        out = ctypes.c_void_p()
        _check(lib.dotpe_load_bank(ctx.handle, ctypes.byref(desc), ctypes.byref(out)))
        self._h = out
        self._keep = []
        self.n_wf, self.n_modes, self.n_bins = n_wf, n_c, n_b
        self.precision = precision
        self.modes = tuple(modes)
        self.layout = layout

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load_library().dotpe_free_bank(self.ctx.handle, self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


FLAG_RERUN_ALL = 1
FLAG_NO_BOUND_PASS = 2


def _event_desc(d, w, det_r, det_D, ext, n_phi, ln_w_ext=None, d_max=5000.0, d0=1.0, n_norm=0.0,
                sub_start=0, sub_count=0, sub_idx=None, cut_delta=0.0, top_k=0, topk_window=40.0,
                stream=None, flags=0, cut_target=0.0, w_dh=None, w_hh=None, dd=0.0):
    """EventDesc over host copies of the inputs; returns (desc, arrays to keep alive).
    With w_dh [K, C, B] and w_hh [K, C, C, B] (relative binning) d and w may be None."""
    keep = []

    def hp(a, dt=np.float64):
        arr, p = _host(a, dt)
        keep.append(arr)
        return arr, p

    if w_dh is not None:
        _, pwdh = hp(np.asarray(w_dh, dtype=np.complex128), np.complex128)
        _, pwhh = hp(np.asarray(w_hh, dtype=np.complex128), np.complex128)
        n_det = np.asarray(w_dh).shape[0]
    else:
        pwdh = pwhh = None
        n_det = np.asarray(d).shape[0]
    pd = hp(np.asarray(d, dtype=np.complex128), np.complex128)[1] if d is not None else None
    pw = hp(w)[1] if w is not None else None
    _, pr = hp(det_r)
    _, pD = hp(det_D)
    n_ext = len(ext["lat"])
    _, plat = hp(ext["lat"])
    _, plon = hp(ext["lon"])
    _, ppsi = hp(ext["psi"])
    _, pci = hp(ext["cos_iota"])
    _, ptg = hp(ext["t_geo"])
    plw = hp(ln_w_ext)[1] if ln_w_ext is not None else None
    psub = None
    if sub_idx is not None:
        si, psub = hp(sub_idx, np.int64)
        sub_count = len(si)
    if stream is not None and not isinstance(stream, int):
        stream = stream.cuda_stream
    desc = EventDesc(n_det, int(n_phi), pd, pw, pr, pD, n_ext, plat, plon, ppsi, pci, ptg,
                     plw, float(d_max), float(d0), float(n_norm), int(sub_start),
                     int(sub_count), psub, float(cut_delta), int(top_k), int(flags),
                     float(topk_window), stream, float(cut_target), pwdh, pwhh, float(dd))
    return desc, keep


def _result(r, arr):
    out = {name: getattr(r, name) for name, _ in EvidenceResult._fields_}
    n = r.topk_count
    out["topk_i"] = np.array([arr[q].i for q in range(n)], dtype=np.int64)
    out["topk_e"] = np.array([arr[q].e for q in range(n)], dtype=np.int64)
    out["topk_lnp"] = np.array([arr[q].ln_p for q in range(n)])
    out["topk_o"] = np.array([arr[q].o_best for q in range(n)], dtype=np.int32)
    # effective sample sizes (eqs. n_effective over pairs, posterior_element, int_ess, ext_ess)
    two = 2.0 * r.ln_sum_p
    out["n_eff_pairs"] = float(np.exp(two - r.ln_sum_p2))
    out["n_eff"] = float(np.exp(two - r.ln_sum_p2_triples))
    out["n_eff_int"] = float(np.exp(two - r.ln_sum_row2))
    out["n_eff_ext"] = float(np.exp(two - r.ln_sum_col2))
    return out


class Event:
    def __init__(self, ctx, bank, **kw):
        lib = load_library()
        self.ctx, self.bank = ctx, bank
        desc, keep = _event_desc(**kw)
        out = ctypes.c_void_p()
        _check(lib.dotpe_set_event(ctx.handle, bank.handle, ctypes.byref(desc), ctypes.byref(out)))
        self._h = out
        self.n_ext = desc.n_ext
        self.n_sub = desc.sub_count if desc.sub_count else bank.n_wf
        self.n_phi = desc.n_phi
        self.n_det = desc.n_det
        self.top_k = desc.top_k

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load_library().dotpe_free_event(self.ctx.handle, self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval_lnl(self, ml=False, triples=False):
        """ln Lbar_ie [n_sub, n_ext] (and max_o lnL^ML, (dh, hh) per triple)."""
        lnl = np.empty((self.n_sub, self.n_ext))
        mlo = np.empty((self.n_sub, self.n_ext)) if ml else None
        tr = np.empty((self.n_sub, self.n_ext, self.n_phi, 2)) if triples else None
        _check(load_library().dotpe_eval_lnl(
            self.ctx.handle, self._h, lnl.ctypes.data, mlo.ctypes.data if ml else None,
            tr.ctypes.data if triples else None, MEM_HOST))
        out = {"lnl": lnl}
        if ml:
            out["ml_max"] = mlo
        if triples:
            out["dh"] = tr[..., 0]
            out["hh"] = tr[..., 1]
        return out

    def eval_lnl_device(self, lnl, ml=None, triples=None):
        """Device-output variant: torch float64 tensors on the GPU."""
        _check(load_library().dotpe_eval_lnl(
            self.ctx.handle, self._h, lnl.data_ptr(), ml.data_ptr() if ml is not None else None,
            triples.data_ptr() if triples is not None else None, MEM_DEVICE))

    def evidence(self):
        r = EvidenceResult()
        k = self.top_k
        arr = (Sample * max(k, 1))()
        _check(load_library().dotpe_evidence(self.ctx.handle, self._h, ctypes.byref(r),
                                             ctypes.cast(arr, ctypes.c_void_p) if k else None))
        return _result(r, arr)

    def sample_posterior(self, n_samples=0, u0=0.5, seed=0, capacity=1 << 20):
        """dotpe_sample_posterior after evidence(): arrays i, e, o, distance, ln_p_pair,
        ln_p_triple of the draws (n_samples <= 0: floor(N_eff / 2))."""
        cap = int(n_samples) if n_samples > 0 else int(capacity)
        arr = (PosteriorSample * cap)()
        n = ctypes.c_int64()
        _check(load_library().dotpe_sample_posterior(self.ctx.handle, self._h, int(n_samples),
                                                     float(u0), ctypes.c_uint64(int(seed)),
                                                     ctypes.cast(arr, ctypes.c_void_p), cap,
                                                     ctypes.byref(n)))
        m = n.value
        out = {name: np.array([getattr(arr[q], name) for q in range(m)])
               for name, _ in PosteriorSample._fields_ if name != "reserved"}
        return out

    def response(self):
        """(R [n_ext, n_det, n_modes] complex, t [n_ext, n_det]) from the device."""
        R = np.empty((self.n_ext, self.n_det, self.bank.n_modes, 2))
        t = np.empty((self.n_ext, self.n_det))
        _check(load_library().dotpe_debug_response(self.ctx.handle, self._h, R.ctypes.data,
                                                    t.ctypes.data))
        return R[..., 0] + 1j * R[..., 1], t

    def bound(self):
        """The bound pass's per-pair bounds on max_o lnL^ML, [2, n_sub, n_ext] float32:
        [0] with the margin of whole rows, [1] with the margin per group and output."""
        out = np.empty((2, self.n_sub, self.n_ext), dtype=np.float32)
        _check(load_library().dotpe_debug_bound(self.ctx.handle, self._h, out.ctypes.data))
        return out


class Server:
    """Continuous admission of events against a resident bank (dotpe_submit /
    dotpe_poll / dotpe_wait); see include/dotpe.h."""

    def __init__(self, ctx, bank, n_slots=4, pool_bytes=0, max_batch=0, batch_pairs=0):
        self.ctx, self.bank = ctx, bank
        h = ctypes.c_void_p()
        desc = ServerDesc(int(n_slots), int(max_batch), int(pool_bytes), int(batch_pairs))
        _check(load_library().dotpe_server_create(ctx.handle, bank.handle, ctypes.byref(desc),
                                                  ctypes.byref(h)))
        self._h = h
        self._top_k = {}

    def event_bytes(self, **kw):
        desc, keep = _event_desc(**kw)
        n = ctypes.c_uint64()
        _check(load_library().dotpe_event_bytes(self.ctx.handle, self.bank.handle,
                                                ctypes.byref(desc), ctypes.byref(n)))
        return int(n.value)

    def submit(self, **kw):
        """Queue an event (same keywords as Context.set_event); returns its ticket."""
        desc, keep = _event_desc(**kw)
        t = ctypes.c_int64()
        _check(load_library().dotpe_submit(self._h, ctypes.byref(desc), ctypes.byref(t)))
        self._top_k[t.value] = desc.top_k
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int32()
        _check(load_library().dotpe_poll(self._h, int(ticket), ctypes.byref(done)))
        return bool(done.value)

    def wait(self, ticket):
        """(result dict as Event.evidence(), timing dict) of a submitted event."""
        r = EvidenceResult()
        info = TicketInfo()
        k = self._top_k.pop(ticket, 0)
        arr = (Sample * max(k, 1))()
        rc = load_library().dotpe_wait(self._h, int(ticket), ctypes.byref(r),
                                       ctypes.cast(arr, ctypes.c_void_p) if k else None,
                                       ctypes.byref(info))
        _check(rc)
        times = {name: getattr(info, name) for name, _ in TicketInfo._fields_}
        return _result(r, arr), times

    def close(self):
        if self._h:
            load_library().dotpe_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

