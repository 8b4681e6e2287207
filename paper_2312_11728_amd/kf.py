"""Python binding of libkf (ctypes).  Argument marshalling only: every step of
the computation runs in the HIP kernels behind the C interface in
include/kf.h; PyTorch supplies device memory and the current stream.

The library is loaded from this directory; if it is missing the import fails
(there is no fallback path)."""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkf.so")

KF_OK, KF_ERR_ARG, KF_ERR_DEVICE, KF_ERR_NOMEM, KF_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
KF_F32, KF_F64 = 0, 1
# per-track status bits (kf_status of include/kf.h)
(KF_TRK_NO_CROSSING, KF_TRK_GRAZING, KF_TRK_NONFINITE, KF_TRK_FP64_FALLBACK, KF_TRK_CHARGE_FLIP, KF_TRK_COV_NOT_PSD,
 KF_TRK_BAD_INPUT, KF_TRK_OUTLIER) = 1, 2, 4, 8, 16, 32, 64, 128
TRK_NO_CROSSING, TRK_GRAZING, TRK_NONFINITE, TRK_FP64_FALLBACK = 1, 2, 4, 8
TRK_CHARGE_FLIP, TRK_COV_NOT_PSD, TRK_BAD_INPUT, TRK_OUTLIER = 16, 32, 64, 128
MAX_LAYERS = 64

EXPORTS = ["kf_create", "kf_destroy", "kf_last_error", "kf_make_seeds", "kf_propagate", "kf_update",
           "kf_fit_tracks", "kf_score_hits", "kf_fit_adjoint", "kf_set_fit_launch", "kf_get_fit_launch",
           "kf_device_cu_count", "kf_reserve", "kf_set_fit_graph",
           "kf_set_kernel_timing", "kf_fit_kernel_time", "kf_seed_fit_tracks", "kf_backward_fit",
           "kf_smooth_tracks", "kf_final_fit", "kf_remove_duplicates", "kf_fit_adjoint_noalloc",
           "kf_propagate_plane", "kf_update_plane", "kf_fit_plane_tracks", "kf_plane_to_global"]

BACKWARD_COV_SCALE = 100.0   # forward covariance scale at the start of the backward fit
FINAL_CHI2_CUT = 30.0        # the final fit's default chi2 cut for one hit
FINAL_MAX_REJECT = 3         # rounds in which the final fit may reject a hit
FINAL_MIN_KEEP = 4           # used hits a track keeps at the least in the final fit

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double


class KfGeometry(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("kind", _vp), ("pos", _vp), ("lo", _vp), ("hi", _vp),
                ("x_over_x0", _vp), ("bz_tesla", _dbl), ("particle_mass_gev", _dbl)]


class KfPlaneGeometry(ctypes.Structure):
    _fields_ = [("n_modules", _i64), ("modules", _vp), ("bz_tesla", _dbl), ("particle_mass_gev", _dbl)]


class KfSearchParams(ctypes.Structure):
    _fields_ = [("beam", ctypes.c_int32), ("chi2_max", ctypes.c_float), ("n_sigma", ctypes.c_float),
                ("hit_bonus", ctypes.c_float), ("miss_penalty", ctypes.c_float), ("max_miss", ctypes.c_int32),
                ("sigma_rphi", ctypes.c_float), ("sigma_z", ctypes.c_float),
                ("win_min_rphi", _vp), ("win_max_rphi", _vp), ("win_min_z", _vp), ("win_max_z", _vp),
                ("reuse_bins", ctypes.c_int32), ("overlap", ctypes.c_int32), ("overlap_bonus", ctypes.c_float)]


class SearchParams:
    """Parameters of kf_score_hits (see kf_search_params in include/kf.h);
    per-layer window limits as arrays of n_layers (cm)."""

    def __init__(self, n_layers, beam=6, chi2_max=30.0, n_sigma=5.0, hit_bonus=10.0, miss_penalty=5.0, max_miss=3,
                 sigma_rphi=0.003, sigma_z=0.01, win_min_rphi=0.01, win_max_rphi=2.0, win_min_z=0.03, win_max_z=2.0,
                 reuse_bins=False, overlap=False, overlap_bonus=5.0):
        self.n_layers = n_layers
        self.beam, self.chi2_max, self.n_sigma = beam, chi2_max, n_sigma
        self.hit_bonus, self.miss_penalty, self.max_miss = hit_bonus, miss_penalty, max_miss
        self.sigma_rphi, self.sigma_z = sigma_rphi, sigma_z
        f = lambda v: np.ascontiguousarray(np.broadcast_to(np.asarray(v, np.float32), (n_layers,)))
        self.win_min_rphi, self.win_max_rphi = f(win_min_rphi), f(win_max_rphi)
        self.win_min_z, self.win_max_z = f(win_min_z), f(win_max_z)
        p = lambda a: a.ctypes.data_as(_vp)
        self.overlap, self.overlap_bonus = bool(overlap), overlap_bonus
        self.struct = KfSearchParams(beam, chi2_max, n_sigma, hit_bonus, miss_penalty, max_miss, sigma_rphi, sigma_z,
                                     p(self.win_min_rphi), p(self.win_max_rphi), p(self.win_min_z),
                                     p(self.win_max_z), int(bool(reuse_bins)), int(bool(overlap)), overlap_bonus)


class KfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libkf error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2312_11728_amd/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    lib.kf_last_error.restype = ctypes.c_char_p
    lib.kf_last_error.argtypes = []
    lib.kf_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
    lib.kf_destroy.argtypes = [_vp]
    lib.kf_make_seeds.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _i64, _vp, _dbl, _i32, _vp, _vp, _vp,
                                  _vp, _vp]
    lib.kf_propagate.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(KfGeometry),
                                 _i32, _vp, _vp, _vp, _vp, _vp]
    lib.kf_update.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.kf_fit_tracks.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp,
                                  ctypes.POINTER(KfGeometry), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _vp, _vp]
    lib.kf_seed_fit_tracks.argtypes = [_vp, ctypes.c_int, _i64, _i64, _i32, _vp, _vp, _vp, _i64, _vp, _vp,
                                       ctypes.POINTER(KfGeometry), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                       _i32, _i32, _vp, _vp]
    lib.kf_backward_fit.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp,
                                    ctypes.POINTER(KfGeometry), _dbl, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.kf_final_fit.argtypes = [_vp, ctypes.c_int, _i64, _i64, _i32, _vp, _vp, _vp, _i64, _vp, _vp,
                                 ctypes.POINTER(KfGeometry), _dbl, _dbl, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                                 _vp, _vp, _vp, _vp]
    lib.kf_remove_duplicates.argtypes = [_vp, _i64, _vp, _i64, _i32, _vp, _i64, ctypes.c_float, _vp, _vp, _vp]
    lib.kf_smooth_tracks.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp,
                                     _vp, ctypes.POINTER(KfGeometry), _dbl, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                     _vp, _vp]
    lib.kf_score_hits.argtypes = [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _i32, ctypes.POINTER(KfGeometry),
                                  ctypes.POINTER(KfSearchParams), _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                  _vp, _vp]
    lib.kf_fit_adjoint.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp,
                                   ctypes.POINTER(KfGeometry), _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.kf_fit_adjoint_noalloc.argtypes = lib.kf_fit_adjoint.argtypes
    pg = ctypes.POINTER(KfPlaneGeometry)
    lib.kf_propagate_plane.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, pg, _i32, _vp, _vp, _vp, _vp,
                                       _vp]
    lib.kf_update_plane.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, pg, _vp, _vp, _vp]
    lib.kf_fit_plane_tracks.argtypes = [_vp, ctypes.c_int, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp,
                                        pg, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.kf_plane_to_global.argtypes = [_vp, ctypes.c_int, _i64, _vp, _vp, pg, _vp, _vp]
    lib.kf_set_fit_launch.argtypes = [_vp, ctypes.c_int, _i32, _i32, _i32, _i32, _i32]
    lib.kf_get_fit_launch.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                      ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
    lib.kf_device_cu_count.argtypes = [_vp, ctypes.POINTER(_i32)]
    lib.kf_reserve.argtypes = [_vp, _i64, _i32]
    lib.kf_set_fit_graph.argtypes = [_vp, _i32]
    lib.kf_set_kernel_timing.argtypes = [_vp, _i32]
    lib.kf_fit_kernel_time.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64)]
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check(rc):
    if rc != KF_OK:
        raise KfError(rc, lib().kf_last_error().decode())


class Geometry:
    """Host-side detector description (kept alive for the C struct)."""

    def __init__(self, kind, pos, lo, hi, x_over_x0, bz=3.8, mass=0.13957):
        self.kind = np.ascontiguousarray(kind, dtype=np.int8)
        self.pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.lo = np.ascontiguousarray(lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(hi, dtype=np.float64)
        self.x_over_x0 = np.ascontiguousarray(x_over_x0, dtype=np.float64)
        self.bz = float(bz)
        self.mass = float(mass)
        self.struct = KfGeometry(self.kind.shape[0], self.kind.ctypes.data, self.pos.ctypes.data,
                                 self.lo.ctypes.data, self.hi.ctypes.data, self.x_over_x0.ctypes.data,
                                 self.bz, self.mass)

    @property
    def n_layers(self):
        return int(self.kind.shape[0])

    @classmethod
    def from_toy(cls, g):
        return cls(g.kind, g.pos, g.lo, g.hi, g.x_over_x0, g.bz, g.mass)


class PlaneGeometry:
    """Tilted-module description: the module table [10, n_modules] (rows cx cy
    cz nx ny nz ux uy uz x_over_x0) copied to the device in one precision, and
    the field; the C struct points at that copy."""

    def __init__(self, modules, bz=3.8, mass=0.13957, dtype=torch.float32, device="cuda"):
        m = torch.as_tensor(np.ascontiguousarray(modules, np.float64))
        if m.dim() != 2 or m.shape[0] != 10 or m.shape[1] < 1:
            raise ValueError(f"modules must have shape [10, M], got {tuple(m.shape)}")
        self.table = m.to(device=device, dtype=dtype).contiguous()
        self.bz = float(bz)
        self.mass = float(mass)
        self.struct = KfPlaneGeometry(self.table.shape[1], self.table.data_ptr(), self.bz, self.mass)

    @property
    def n_modules(self):
        return int(self.table.shape[1])

    @property
    def dtype(self):
        return self.table.dtype

    @classmethod
    def from_toy(cls, g, dtype=torch.float32, device="cuda"):
        return cls(g.modules, g.bz, g.mass, dtype=dtype, device=device)


def _need_plane(geom, dt, dev):
    if not isinstance(geom, PlaneGeometry):
        raise TypeError("geom must be a PlaneGeometry")
    if geom.table.dtype != dt or geom.table.device != dev:
        raise ValueError(f"the module table is {geom.table.dtype} on {geom.table.device}, expected {dt} on {dev}")
    return geom


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def _prec(dtype):
    if dtype == torch.float32:
        return KF_F32
    if dtype == torch.float64:
        return KF_F64
    raise TypeError(f"unsupported dtype {dtype}")


def _need(t, name, dtype=None, dev=None, rows=None):
    if not torch.is_tensor(t):
        raise TypeError(f"{name} must be a torch tensor")
    if dev is not None and t.device != dev:
        raise ValueError(f"{name} is on {t.device}, expected {dev}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if rows is not None and (t.dim() != 2 or t.shape[0] != rows):
        raise ValueError(f"{name} must have shape [{rows}, N], got {tuple(t.shape)}")
    return t


def _need_offsets(hit_offsets, n, dev):
    """CSR offsets of n tracks: int32 [n + 1] on the device."""
    _need(hit_offsets, "hit_offsets", torch.int32, dev)
    if hit_offsets.dim() != 1 or hit_offsets.numel() != n + 1:
        raise ValueError(f"hit_offsets must hold n + 1 = {n + 1} entries, got {tuple(hit_offsets.shape)}")
    return hit_offsets


def _stream(dev):
    return _vp(torch.cuda.current_stream(dev).cuda_stream)


class Context:
    """One libkf context on one device (re-entrant: no global state)."""

    def __init__(self, device=0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = _vp()
        _check(lib().kf_create(ctypes.byref(h), self.device.index or 0))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().kf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, max_tracks, max_len=26):
        """Workspace for the packed hit layout of fit_tracks (see kf_reserve)."""
        _check(lib().kf_reserve(self.handle, int(max_tracks), int(max_len)))

    # ---- tuning -----------------------------------------------------------
    def set_fit_launch(self, dtype, block, persistent, blocks_per_cu, waves=1, layout=0):
        _check(lib().kf_set_fit_launch(self.handle, _prec(dtype), block, persistent, blocks_per_cu, waves, layout))

    def set_kernel_timing(self, max_launches):
        """Record HIP events around the fit kernel of the next `max_launches`
        fit_tracks calls (0 turns it off; see kf_set_kernel_timing)."""
        _check(lib().kf_set_kernel_timing(self.handle, int(max_launches)))

    def fit_kernel_time(self):
        """(total ms, launches, dropped) of the fit kernels recorded since the
        last query; waits for them."""
        ms, n, d = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().kf_fit_kernel_time(self.handle, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(d)))
        return ms.value, n.value, d.value

    def set_fit_graph(self, enable=True):
        """Replay kf_fit_tracks from a captured hipGraph (see kf_set_fit_graph)."""
        _check(lib().kf_set_fit_graph(self.handle, int(bool(enable))))

    def get_fit_launch(self, dtype):
        b, p, k, w, l = _i32(), _i32(), _i32(), _i32(), _i32()
        _check(lib().kf_get_fit_launch(self.handle, _prec(dtype), ctypes.byref(b), ctypes.byref(p), ctypes.byref(k),
                                       ctypes.byref(w), ctypes.byref(l)))
        return b.value, p.value, k.value, w.value, l.value

    def cu_count(self):
        n = _i32()
        _check(lib().kf_device_cu_count(self.handle, ctypes.byref(n)))
        return n.value

    # ---- entry points -----------------------------------------------------
    def make_seeds(self, hit_offsets, hit_valid, hit_pos, bz, mode=0, out=None):
        dev = self.device
        _need(hit_offsets, "hit_offsets", torch.int32, dev)
        if hit_offsets.dim() != 1 or hit_offsets.numel() < 1:
            raise ValueError("hit_offsets must be a 1-D tensor of n + 1 entries")
        n = hit_offsets.shape[0] - 1
        _need(hit_valid, "hit_valid", torch.uint8, dev)
        _need(hit_pos, "hit_pos", None, dev, rows=3)
        dt = hit_pos.dtype
        if out is None:
            out = (torch.empty(6, n, dtype=dt, device=dev), torch.empty(21, n, dtype=dt, device=dev),
                   torch.empty(n, dtype=torch.int8, device=dev), torch.empty(n, dtype=torch.int32, device=dev))
        st, cov, q, status = out
        _check(lib().kf_make_seeds(self.handle, _prec(dt), n, st.stride(0), _ptr(hit_offsets), _ptr(hit_valid),
                                   hit_pos.shape[1], _ptr(hit_pos), float(bz), int(mode), _ptr(st), _ptr(cov),
                                   _ptr(q), _ptr(status), _stream(dev)))
        return st, cov, q, status

    def propagate(self, state, cov, charge, target_layer, geom: Geometry, from_layer=None, apply_material=True,
                  status=None):
        dev = self.device
        dt = state.dtype
        n = state.shape[1]
        _need(state, "state", dt, dev, rows=6)
        _need(cov, "cov", dt, dev, rows=21)
        _need(charge, "charge", torch.int8, dev)
        _need(target_layer, "target_layer", torch.int16, dev)
        if from_layer is not None:
            _need(from_layer, "from_layer", torch.int16, dev)
        so = torch.empty_like(state)
        co = torch.empty_like(cov)
        path = torch.empty(n, dtype=dt, device=dev)
        if status is None:
            status = torch.zeros(n, dtype=torch.int32, device=dev)
        _check(lib().kf_propagate(self.handle, _prec(dt), n, state.stride(0), _ptr(state), _ptr(cov), _ptr(charge),
                                  _ptr(target_layer), _ptr(from_layer), ctypes.byref(geom.struct),
                                  int(bool(apply_material)), _ptr(so), _ptr(co), _ptr(path), _ptr(status),
                                  _stream(dev)))
        return so, co, path, status

    def update(self, state, cov, charge, hit_pos, hit_cov, status=None):
        """In-place update of state/cov/charge; returns (chi2, status)."""
        dev = self.device
        dt = state.dtype
        n = state.shape[1]
        _need(state, "state", dt, dev, rows=6)
        _need(cov, "cov", dt, dev, rows=21)
        _need(charge, "charge", torch.int8, dev)
        _need(hit_pos, "hit_pos", dt, dev, rows=3)
        _need(hit_cov, "hit_cov", dt, dev, rows=6)
        chi2 = torch.empty(n, dtype=dt, device=dev)
        if status is None:
            status = torch.zeros(n, dtype=torch.int32, device=dev)
        _check(lib().kf_update(self.handle, _prec(dt), n, state.stride(0), _ptr(state), _ptr(cov), _ptr(charge),
                               _ptr(hit_pos), _ptr(hit_cov), _ptr(chi2), _ptr(status), _stream(dev)))
        return chi2, status

    # ---- tilted planar modules ---------------------------------------------
    def propagate_plane(self, state, cov, charge, target_module, geom: PlaneGeometry, apply_material=True,
                        status=None):
        dev = self.device
        dt = state.dtype
        n = state.shape[1]
        _need(state, "state", dt, dev, rows=6)
        _need(cov, "cov", dt, dev, rows=21)
        _need(charge, "charge", torch.int8, dev)
        _need(target_module, "target_module", torch.int32, dev)
        _need_plane(geom, dt, dev)
        so = torch.empty_like(state)
        co = torch.empty_like(cov)
        path = torch.empty(n, dtype=dt, device=dev)
        if status is None:
            status = torch.zeros(n, dtype=torch.int32, device=dev)
        _check(lib().kf_propagate_plane(self.handle, _prec(dt), n, state.stride(0), _ptr(state), _ptr(cov),
                                        _ptr(charge), _ptr(target_module), ctypes.byref(geom.struct),
                                        int(bool(apply_material)), _ptr(so), _ptr(co), _ptr(path), _ptr(status),
                                        _stream(dev)))
        return so, co, path, status

    def update_plane(self, state, cov, charge, module, hit_uv, hit_cov_uv, geom: PlaneGeometry, status=None):
        """In-place local update of state/cov/charge; returns (chi2, status)."""
        dev = self.device
        dt = state.dtype
        n = state.shape[1]
        _need(state, "state", dt, dev, rows=6)
        _need(cov, "cov", dt, dev, rows=21)
        _need(charge, "charge", torch.int8, dev)
        _need(module, "module", torch.int32, dev)
        _need(hit_uv, "hit_uv", dt, dev, rows=2)
        _need(hit_cov_uv, "hit_cov_uv", dt, dev, rows=3)
        _need_plane(geom, dt, dev)
        chi2 = torch.empty(n, dtype=dt, device=dev)
        if status is None:
            status = torch.zeros(n, dtype=torch.int32, device=dev)
        _check(lib().kf_update_plane(self.handle, _prec(dt), n, state.stride(0), _ptr(state), _ptr(cov), _ptr(charge),
                                     _ptr(module), _ptr(hit_uv), _ptr(hit_cov_uv), ctypes.byref(geom.struct),
                                     _ptr(chi2), _ptr(status), _stream(dev)))
        return chi2, status

    def fit_plane_tracks(self, seed_state, seed_cov, seed_charge, hit_offsets, hit_module, hit_valid, hit_uv,
                         hit_cov_uv, geom: PlaneGeometry, out=None):
        dev = self.device
        dt = seed_state.dtype
        n = seed_state.shape[1]
        _need(seed_state, "seed_state", dt, dev, rows=6)
        _need(seed_cov, "seed_cov", dt, dev, rows=21)
        _need(seed_charge, "seed_charge", torch.int8, dev)
        _need_offsets(hit_offsets, n, dev)
        _need(hit_module, "hit_module", torch.int32, dev)
        _need(hit_valid, "hit_valid", torch.uint8, dev)
        _need(hit_uv, "hit_uv", dt, dev, rows=2)
        _need(hit_cov_uv, "hit_cov_uv", dt, dev, rows=3)
        _need_plane(geom, dt, dev)
        if out is None:
            out = fit_outputs(n, dt, dev)
        _need_outputs(out, n, dt, dev)
        _check(lib().kf_fit_plane_tracks(self.handle, _prec(dt), n, seed_state.stride(0), _ptr(seed_state),
                                         _ptr(seed_cov), _ptr(seed_charge), _ptr(hit_offsets), _ptr(hit_module),
                                         _ptr(hit_valid), hit_uv.shape[1], _ptr(hit_uv), _ptr(hit_cov_uv),
                                         ctypes.byref(geom.struct), _ptr(out["state"]), _ptr(out["cov"]),
                                         _ptr(out["charge"]), _ptr(out["chi2"]), _ptr(out["ndf"]), _ptr(out["status"]),
                                         _stream(dev)))
        return out

    def plane_to_global(self, module, hit_uv, geom: PlaneGeometry, out=None):
        """Global positions [3, n_hits] of local hits (module, hit_uv [2, n_hits])."""
        dev = self.device
        dt = hit_uv.dtype
        _need(module, "module", torch.int32, dev)
        _need(hit_uv, "hit_uv", dt, dev, rows=2)
        _need_plane(geom, dt, dev)
        nh = hit_uv.shape[1]
        if module.numel() != nh:
            raise ValueError(f"module holds {module.numel()} entries, hit_uv {nh}")
        if out is None:
            out = torch.empty(3, nh, dtype=dt, device=dev)
        _need(out, "out", dt, dev, rows=3)
        _check(lib().kf_plane_to_global(self.handle, _prec(dt), nh, _ptr(module), _ptr(hit_uv),
                                        ctypes.byref(geom.struct), _ptr(out), _stream(dev)))
        return out

    def fit_tracks(self, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov,
                   geom: Geometry, align=None, checkpoints=None, seg=1, max_len=26, out=None):
        dev = self.device
        dt = seed_state.dtype
        n = seed_state.shape[1]
        _need(seed_state, "seed_state", dt, dev, rows=6)
        _need(seed_cov, "seed_cov", dt, dev, rows=21)
        _need(seed_charge, "seed_charge", torch.int8, dev)
        _need_offsets(hit_offsets, n, dev)
        _need(hit_layer, "hit_layer", torch.int16, dev)
        _need(hit_valid, "hit_valid", torch.uint8, dev)
        _need(hit_pos, "hit_pos", dt, dev, rows=3)
        _need(hit_cov, "hit_cov", dt, dev, rows=6)
        if align is not None:
            _need(align, "align", dt, dev, rows=2)
        if checkpoints is not None:
            _need(checkpoints, "checkpoints", dt, dev, rows=28)
        if out is None:
            out = fit_outputs(n, dt, dev)
        _need_outputs(out, n, dt, dev)
        _check(lib().kf_fit_tracks(self.handle, _prec(dt), n, seed_state.stride(0), _ptr(seed_state), _ptr(seed_cov),
                                   _ptr(seed_charge), _ptr(hit_offsets), _ptr(hit_layer), _ptr(hit_valid),
                                   hit_pos.shape[1], _ptr(hit_pos), _ptr(hit_cov), ctypes.byref(geom.struct),
                                   _ptr(align), _ptr(out["state"]), _ptr(out["cov"]), _ptr(out["charge"]),
                                   _ptr(out["chi2"]), _ptr(out["ndf"]), _ptr(checkpoints), int(seg), int(max_len),
                                   _ptr(out["status"]), _stream(dev)))
        return out


    def backward_fit(self, fwd, hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov, geom: Geometry,
                     cov_scale=BACKWARD_COV_SCALE, max_len=26, out=None, use_status=True):
        """Backward fit (kf_backward_fit) from a forward fit's outputs `fwd`
        (state [6, n], cov [21, n], charge [n], status [n] as fit_tracks
        returns them; status is passed unless use_status is False).  Returns
        the outputs of fit_tracks' form, on each track's first valid entry."""
        dev = self.device
        st_in, cov_in, q_in = fwd["state"], fwd["cov"], fwd["charge"]
        dt = st_in.dtype
        n = st_in.shape[1]
        _need(st_in, "state", dt, dev, rows=6)
        _need(cov_in, "cov", dt, dev, rows=21)
        _need(q_in, "charge", torch.int8, dev)
        _need_offsets(hit_offsets, n, dev)
        _need(hit_layer, "hit_layer", torch.int16, dev)
        _need(hit_valid, "hit_valid", torch.uint8, dev)
        _need(hit_pos, "hit_pos", dt, dev, rows=3)
        _need(hit_cov, "hit_cov", dt, dev, rows=6)
        status = fwd["status"] if use_status else None
        if status is not None:
            _need(status, "status", torch.int32, dev)
        if st_in.stride(0) != n or cov_in.stride(0) != n:
            raise ValueError("state and cov must have leading dimension n (the outputs are [rows, n])")
        if out is None:
            out = fit_outputs(n, dt, dev)
        _need_outputs(out, n, dt, dev)
        _check(lib().kf_backward_fit(self.handle, _prec(dt), n, st_in.stride(0), _ptr(st_in), _ptr(cov_in), _ptr(q_in),
                                     _ptr(status), _ptr(hit_offsets), _ptr(hit_layer), _ptr(hit_valid),
                                     hit_pos.shape[1], _ptr(hit_pos), _ptr(hit_cov), ctypes.byref(geom.struct),
                                     float(cov_scale), int(max_len), _ptr(out["state"]), _ptr(out["cov"]),
                                     _ptr(out["charge"]), _ptr(out["chi2"]), _ptr(out["ndf"]), _ptr(out["status"]),
                                     _stream(dev)))
        return out

    def final_fit(self, hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov, geom: Geometry, seed_mode=0,
                  chi2_cut=FINAL_CHI2_CUT, max_reject=FINAL_MAX_REJECT, min_keep=FINAL_MIN_KEEP,
                  cov_scale=BACKWARD_COV_SCALE, max_len=26, out=None, outlier=None, hit_chi2=None,
                  want_hit_chi2=True):
        """Final fit with outlier rejection (kf_final_fit): rounds of seeding,
        forward fit and smoothing backward fit over each track's used hits,
        rejecting the hit with the worst unbiased chi2 above chi2_cut.
        Returns (out, outlier, hit_chi2): fit_tracks-form outputs (the
        backward fit's state on each track's first used entry), the uint8
        mask [n_hits] of rejected entries and the per-hit unbiased chi2
        [n_hits] (None unless want_hit_chi2 or given)."""
        dev = self.device
        dt = hit_pos.dtype
        _need(hit_offsets, "hit_offsets", torch.int32, dev)
        if hit_offsets.dim() != 1 or hit_offsets.numel() < 1:
            raise ValueError("hit_offsets must be a 1-D tensor of n + 1 entries")
        n = hit_offsets.shape[0] - 1
        _need(hit_layer, "hit_layer", torch.int16, dev)
        _need(hit_valid, "hit_valid", torch.uint8, dev)
        _need(hit_pos, "hit_pos", dt, dev, rows=3)
        _need(hit_cov, "hit_cov", dt, dev, rows=6)
        n_hits = hit_pos.shape[1]
        if out is None:
            out = fit_outputs(n, dt, dev)
        _need_outputs(out, n, dt, dev)
        if outlier is None:
            outlier = torch.empty(n_hits, dtype=torch.uint8, device=dev)
        _need(outlier, "outlier", torch.uint8, dev)
        if outlier.numel() < n_hits:
            raise ValueError(f"outlier must hold n_hits = {n_hits} entries")
        if hit_chi2 is None and want_hit_chi2:
            hit_chi2 = torch.full((n_hits,), float("nan"), dtype=dt, device=dev)
        if hit_chi2 is not None:
            _need(hit_chi2, "hit_chi2", dt, dev)
            if hit_chi2.numel() < n_hits:
                raise ValueError(f"hit_chi2 must hold n_hits = {n_hits} entries")
        _check(lib().kf_final_fit(self.handle, _prec(dt), n, n, int(seed_mode), _ptr(hit_offsets), _ptr(hit_layer),
                                  _ptr(hit_valid), n_hits, _ptr(hit_pos), _ptr(hit_cov), ctypes.byref(geom.struct),
                                  float(cov_scale), float(chi2_cut), int(max_reject), int(min_keep), int(max_len),
                                  _ptr(out["state"]), _ptr(out["cov"]), _ptr(out["charge"]), _ptr(out["chi2"]),
                                  _ptr(out["ndf"]), _ptr(out["status"]), _ptr(outlier), _ptr(hit_chi2),
                                  _stream(dev)))
        return out, outlier, hit_chi2

    def remove_duplicates(self, track_hits, score, frac=0.5, keep=None, dup_of=None):
        """Duplicate removal (kf_remove_duplicates) over n tracks:
        track_hits int32 [n, L] or a view with unit stride along L (e.g. the
        rank-0 slice cand_hits[:, 0, :] of score_hits), score float32 [n]
        (strided views allowed).  Returns (keep uint8 [n], dup_of int32 [n])."""
        dev = self.device
        if track_hits.dtype != torch.int32 or track_hits.dim() != 2 or track_hits.stride(1) != 1:
            raise ValueError("track_hits must be int32 [n, L] with unit stride along L")
        if score.dtype != torch.float32 or score.dim() != 1:
            raise ValueError("score must be float32 [n]")
        n, L = track_hits.shape
        if score.shape[0] != n:
            raise ValueError("score and track_hits disagree on n")
        if track_hits.device != dev or score.device != dev:
            raise ValueError("inputs must be on the context's device")
        if keep is None:
            keep = torch.empty(n, dtype=torch.uint8, device=dev)
        if dup_of is None:
            dup_of = torch.empty(n, dtype=torch.int32, device=dev)
        _need(keep, "keep", torch.uint8, dev)
        _need(dup_of, "dup_of", torch.int32, dev)
        if keep.numel() < n or dup_of.numel() < n:
            raise ValueError(f"keep and dup_of must hold n = {n} entries")
        _check(lib().kf_remove_duplicates(self.handle, n, _ptr(track_hits), max(track_hits.stride(0), L), L,
                                          _ptr(score), max(score.stride(0), 1), float(frac), _ptr(keep),
                                          _ptr(dup_of), _stream(dev)))
        return keep, dup_of

    def smooth_tracks(self, fwd, checkpoints, hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov, geom: Geometry,
                      cov_scale=BACKWARD_COV_SCALE, max_len=26, out=None, smooth=None, use_status=True):
        """Backward fit with smoothing (kf_smooth_tracks): `fwd` and
        `checkpoints` from fit_tracks / seed_fit_tracks called with
        checkpoints=[28, n * (max_len - 1)], seg=1 and the same max_len.
        Returns (out, smooth): the backward fit's outputs, and the smoothed
        state [6, max_len, n] and covariance [21, max_len, n] of entry r of
        track t at [:, r, t] (entries not smoothed are not written; smooth
        may pass preallocated tensors)."""
        dev = self.device
        st_in, cov_in, q_in = fwd["state"], fwd["cov"], fwd["charge"]
        dt = st_in.dtype
        n = st_in.shape[1]
        for t_, nm, rows in ((st_in, "state", 6), (cov_in, "cov", 21), (hit_pos, "hit_pos", 3), (hit_cov, "hit_cov", 6),
                             (checkpoints, "checkpoints", 28)):
            _need(t_, nm, dt, dev, rows=rows)
        _need(q_in, "charge", torch.int8, dev)
        _need_offsets(hit_offsets, n, dev)
        _need(hit_layer, "hit_layer", torch.int16, dev)
        _need(hit_valid, "hit_valid", torch.uint8, dev)
        if st_in.stride(0) != n or cov_in.stride(0) != n:
            raise ValueError("state and cov must have leading dimension n")
        if checkpoints.shape[1] != n * max(1, max_len - 1):
            raise ValueError("checkpoints must be [28, n * (max_len - 1)] (seg = 1)")
        status = fwd["status"] if use_status else None
        if status is not None:
            _need(status, "status", torch.int32, dev)
            if status.numel() != n:
                raise ValueError(f"status must hold n = {n} entries")
        if out is None:
            out = fit_outputs(n, dt, dev)
        _need_outputs(out, n, dt, dev)
        if smooth is None:
            smooth = dict(state=torch.full((6, max_len, n), float("nan"), dtype=dt, device=dev),
                          cov=torch.full((21, max_len, n), float("nan"), dtype=dt, device=dev))
        for k, rows in (("state", 6), ("cov", 21)):
            s_ = smooth.get(k) if isinstance(smooth, dict) else None
            if (not torch.is_tensor(s_) or tuple(s_.shape) != (rows, max_len, n) or s_.dtype != dt
                    or s_.device != dev or not s_.is_contiguous()):
                raise ValueError(f"smooth[{k!r}] must be a contiguous [{rows}, {max_len}, {n}] tensor of {dt} on {dev}")
        _check(lib().kf_smooth_tracks(self.handle, _prec(dt), n, n, _ptr(st_in), _ptr(cov_in), _ptr(q_in),
                                      _ptr(status), _ptr(checkpoints), _ptr(hit_offsets), _ptr(hit_layer),
                                      _ptr(hit_valid), hit_pos.shape[1], _ptr(hit_pos), _ptr(hit_cov),
                                      ctypes.byref(geom.struct), float(cov_scale), int(max_len), _ptr(out["state"]),
                                      _ptr(out["cov"]), _ptr(out["charge"]), _ptr(out["chi2"]), _ptr(out["ndf"]),
                                      _ptr(out["status"]), _ptr(smooth["state"]), _ptr(smooth["cov"]), _stream(dev)))
        return out, smooth

    def seed_fit_tracks(self, hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov, geom: Geometry, seed_mode,
                        align=None, seeds=None, checkpoints=None, seg=1, max_len=26, out=None):
        """Seeding and fit in one launch (kf_seed_fit_tracks).  seeds: None,
        or a (state [6, n], cov [21, n], charge [n]) triple of device tensors
        that receive the seeds.  Returns the fit outputs as fit_tracks does;
        status holds the seeding and the fit bits."""
        dev = self.device
        dt = hit_pos.dtype
        _need(hit_offsets, "hit_offsets", torch.int32, dev)
        if hit_offsets.dim() != 1 or hit_offsets.numel() < 1:
            raise ValueError("hit_offsets must be a 1-D tensor of n + 1 entries")
        n = hit_offsets.shape[0] - 1
        _need(hit_layer, "hit_layer", torch.int16, dev)
        _need(hit_valid, "hit_valid", torch.uint8, dev)
        _need(hit_pos, "hit_pos", dt, dev, rows=3)
        _need(hit_cov, "hit_cov", dt, dev, rows=6)
        if align is not None:
            _need(align, "align", dt, dev, rows=2)
        if checkpoints is not None:
            _need(checkpoints, "checkpoints", dt, dev, rows=28)
        ss = sc = sq = None
        if seeds is not None:
            ss, sc, sq = seeds
            _need(ss, "seed_state", dt, dev, rows=6)
            _need(sc, "seed_cov", dt, dev, rows=21)
            _need(sq, "seed_charge", torch.int8, dev)
            if ss.stride(0) != n or sc.stride(0) != n:
                raise ValueError("seed outputs must have leading dimension n")
        if out is None:
            out = fit_outputs(n, dt, dev)
        _need_outputs(out, n, dt, dev)
        _check(lib().kf_seed_fit_tracks(self.handle, _prec(dt), n, n, int(seed_mode), _ptr(hit_offsets),
                                        _ptr(hit_layer), _ptr(hit_valid), hit_pos.shape[1], _ptr(hit_pos),
                                        _ptr(hit_cov), ctypes.byref(geom.struct), _ptr(align), _ptr(ss), _ptr(sc),
                                        _ptr(sq), _ptr(out["state"]), _ptr(out["cov"]), _ptr(out["charge"]),
                                        _ptr(out["chi2"]), _ptr(out["ndf"]), _ptr(checkpoints), int(seg),
                                        int(max_len), _ptr(out["status"]), _stream(dev)))
        return out

    def score_hits(self, seed_state, seed_cov, seed_charge, seed_layer, layer_plan, geom: Geometry,
                   params: SearchParams, pool_layer_offsets, pool_pos, pool_cov, pool_hit_id, want_state=True,
                   pool_module=None, want_overlap=False):
        """Combinatorial candidate search (kf_score_hits, FP32).  layer_plan and
        pool_layer_offsets are host sequences; the rest device tensors
        (pool_module: int32 [n_pool], needed with params.overlap).
        Returns (hits [n, beam, plan_len] int32, score [n, beam], state
        [6, n * beam] or None, status [n]), and with want_overlap the overlap
        hits [n, beam, plan_len] int32 as a fifth element."""
        dev = self.device
        n = seed_state.shape[1]
        _need(seed_state, "seed_state", torch.float32, dev, rows=6)
        _need(seed_cov, "seed_cov", torch.float32, dev, rows=21)
        _need(seed_charge, "seed_charge", torch.int8, dev)
        _need(seed_layer, "seed_layer", torch.int16, dev)
        _need(pool_pos, "pool_pos", torch.float32, dev, rows=3)
        _need(pool_cov, "pool_cov", torch.float32, dev, rows=6)
        _need(pool_hit_id, "pool_hit_id", torch.int32, dev)
        if pool_module is not None:
            _need(pool_module, "pool_module", torch.int32, dev)
            if pool_module.numel() != pool_hit_id.numel():
                raise ValueError("pool_module must hold one module id per pool hit")
        plan = np.ascontiguousarray(np.asarray(layer_plan, np.int16))
        off = np.ascontiguousarray(np.asarray(pool_layer_offsets, np.int32))
        B, P = params.beam, plan.shape[0]
        hits = torch.empty(n, B, P, dtype=torch.int32, device=dev)
        score = torch.empty(n, B, dtype=torch.float32, device=dev)
        state = torch.empty(6, n * B, dtype=torch.float32, device=dev) if want_state else None
        status = torch.empty(n, dtype=torch.int32, device=dev)
        ovl = torch.empty(n, B, P, dtype=torch.int32, device=dev) if want_overlap else None
        _check(lib().kf_score_hits(self.handle, n, seed_state.stride(0), _ptr(seed_state), _ptr(seed_cov),
                                   _ptr(seed_charge), _ptr(seed_layer), plan.ctypes.data_as(_vp), P,
                                   ctypes.byref(geom.struct), ctypes.byref(params.struct), off.ctypes.data_as(_vp),
                                   pool_pos.shape[1], _ptr(pool_pos), _ptr(pool_cov), _ptr(pool_hit_id),
                                   _ptr(pool_module), _ptr(hits), _ptr(ovl), _ptr(score), _ptr(state), _ptr(status),
                                   _stream(dev)))
        return (hits, score, state, status, ovl) if want_overlap else (hits, score, state, status)

    def fit_adjoint(self, seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov,
                    geom: Geometry, checkpoints, seg, max_len, fwd_status, align=None, dL_dchi2=None,
                    want_align=True, no_alloc=False, out=None):
        """Reverse pass of fit_tracks (kf_fit_adjoint): returns (grad_seed [6, n],
        grad_hit_pos [3, n_hits], grad_align [2, n_layers] or None).  The inputs,
        seg and max_len must be those of the fit_tracks call that wrote
        `checkpoints` and `fwd_status`.  no_alloc: call kf_fit_adjoint_noalloc
        (the library's fixed scratch instead of its growing workspace).  out:
        None, or a (grad_seed, grad_hit_pos, grad_align or None) triple of
        preallocated tensors of those shapes."""
        dev = self.device
        dt = seed_state.dtype
        n = seed_state.shape[1]
        _need(seed_state, "seed_state", dt, dev, rows=6)
        _need(seed_cov, "seed_cov", dt, dev, rows=21)
        _need(seed_charge, "seed_charge", torch.int8, dev)
        _need_offsets(hit_offsets, n, dev)
        _need(hit_layer, "hit_layer", torch.int16, dev)
        _need(hit_valid, "hit_valid", torch.uint8, dev)
        _need(hit_pos, "hit_pos", dt, dev, rows=3)
        _need(hit_cov, "hit_cov", dt, dev, rows=6)
        _need(checkpoints, "checkpoints", dt, dev, rows=28)
        _need(fwd_status, "fwd_status", torch.int32, dev)
        if align is not None:
            _need(align, "align", dt, dev, rows=2)
        if dL_dchi2 is not None:
            _need(dL_dchi2, "dL_dchi2", dt, dev)
        if out is None:
            gs = torch.empty(6, n, dtype=dt, device=dev)
            gh = torch.empty(3, hit_pos.shape[1], dtype=dt, device=dev)
            ga = torch.empty(2, geom.n_layers, dtype=dt, device=dev) if want_align else None
        else:
            gs, gh, ga = out
            _need(gs, "grad_seed", dt, dev, rows=6)
            _need(gh, "grad_hit_pos", dt, dev, rows=3)
            if gs.shape[1] != n or gh.shape[1] != hit_pos.shape[1]:
                raise ValueError("grad_seed must be [6, n] and grad_hit_pos [3, n_hits]")
            if ga is not None:
                _need(ga, "grad_align", dt, dev, rows=2)
                if ga.shape[1] != geom.n_layers:
                    raise ValueError("grad_align must be [2, n_layers]")
        fn = lib().kf_fit_adjoint_noalloc if no_alloc else lib().kf_fit_adjoint
        _check(fn(self.handle, _prec(dt), n, seed_state.stride(0), _ptr(seed_state),
                                    _ptr(seed_cov), _ptr(seed_charge), _ptr(hit_offsets), _ptr(hit_layer),
                                    _ptr(hit_valid), hit_pos.shape[1], _ptr(hit_pos), _ptr(hit_cov),
                                    ctypes.byref(geom.struct), _ptr(align), _ptr(checkpoints), int(seg),
                                    int(max_len), _ptr(dL_dchi2), _ptr(gs), _ptr(gh), _ptr(ga), _ptr(fwd_status),
                                    _stream(dev)))
        return gs, gh, ga


class KfFit(torch.autograd.Function):
    """chi2 of the forward fit as a differentiable function of the seed states
    [6, n], the hit positions [3, n_hits] and the alignment offsets
    [2, n_layers]: forward = kf_fit_tracks with checkpoints every `seg` entries,
    backward = kf_fit_adjoint (the states are recomputed from the checkpoints).
    The other inputs are constants.  Returns (chi2 [n], state, cov, charge, ndf,
    status) as fit_tracks does; only chi2 carries a gradient."""

    @staticmethod
    def forward(fctx, seed_state, hit_pos, align, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, hit_cov,
                geom, kctx, seg, max_len):
        n = seed_state.shape[1]
        ck = torch.empty(28, n * n_checkpoint_segments(max_len, seg), dtype=seed_state.dtype,
                         device=seed_state.device)
        out = kctx.fit_tracks(seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, hit_pos,
                              hit_cov, geom, align=align, checkpoints=ck, seg=seg, max_len=max_len)
        fctx.save_for_backward(seed_state, hit_pos, align if align is not None else torch.empty(0), seed_cov,
                               seed_charge, hit_offsets, hit_layer, hit_valid, hit_cov, ck, out["status"])
        fctx.has_align = align is not None
        fctx.geom, fctx.kctx, fctx.seg, fctx.max_len = geom, kctx, seg, max_len
        rest = (out["state"], out["cov"], out["charge"], out["ndf"], out["status"])
        fctx.mark_non_differentiable(*rest)
        return (out["chi2"],) + rest

    @staticmethod
    def backward(fctx, g_chi2, *unused):
        (seed_state, hit_pos, align, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, hit_cov, ck,
         status) = fctx.saved_tensors
        al = align if fctx.has_align else None
        want_align = fctx.needs_input_grad[2]
        gs, gh, ga = fctx.kctx.fit_adjoint(seed_state, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid,
                                           hit_pos, hit_cov, fctx.geom, ck, fctx.seg, fctx.max_len, status,
                                           align=al, dL_dchi2=g_chi2.contiguous(), want_align=want_align)
        return (gs, gh, ga if want_align else None) + (None,) * 10


def fit_chi2(kctx, seed_state, hit_pos, align, seed_cov, seed_charge, hit_offsets, hit_layer, hit_valid, hit_cov,
             geom, seg=5, max_len=26):
    """Differentiable fit (see KfFit); returns (chi2, fit outputs dict)."""
    chi2, state, cov, charge, ndf, status = KfFit.apply(seed_state, hit_pos, align, seed_cov, seed_charge,
                                                        hit_offsets, hit_layer, hit_valid, hit_cov, geom, kctx, seg,
                                                        max_len)
    return chi2, dict(state=state, cov=cov, charge=charge, chi2=chi2.detach(), ndf=ndf, status=status)


def fit_outputs(n, dtype, device):
    return dict(state=torch.empty(6, n, dtype=dtype, device=device), cov=torch.empty(21, n, dtype=dtype, device=device),
                charge=torch.empty(n, dtype=torch.int8, device=device), chi2=torch.empty(n, dtype=dtype, device=device),
                ndf=torch.empty(n, dtype=torch.int32, device=device), status=torch.empty(n, dtype=torch.int32, device=device))


def _need_outputs(out, n, dtype, device):
    """The caller's output dict has the shapes and types fit_outputs makes."""
    spec = (("state", 6, dtype), ("cov", 21, dtype), ("charge", 0, torch.int8), ("chi2", 0, dtype),
            ("ndf", 0, torch.int32), ("status", 0, torch.int32))
    for k, rows, dt in spec:
        t = out.get(k) if isinstance(out, dict) else None
        shape = (rows, n) if rows else (n,)
        if t is None or t.dtype != dt or t.device != device or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"out[{k!r}] must be a contiguous {list(shape)} tensor of {dt} on {device}")


def n_checkpoint_segments(max_len, seg):
    return max(1, (max_len - 1 + seg - 1) // seg)


def event_tensors(ev, dtype=torch.float32, device="cuda"):
    """Device copies of a batch in the CSR / SoA layout of the interface
    (hit_pos [3][n_hits], hit_cov [6][n_hits], hit_offsets [n+1], ...)."""
    dev = torch.device(device)
    return dict(
        hit_offsets=torch.as_tensor(np.ascontiguousarray(ev.hit_offsets, np.int32), device=dev),
        hit_layer=torch.as_tensor(np.ascontiguousarray(ev.hit_layer, np.int16), device=dev),
        hit_valid=torch.as_tensor(np.ascontiguousarray(ev.hit_valid, np.uint8), device=dev),
        hit_pos=torch.as_tensor(np.ascontiguousarray(ev.hit_pos), device=dev).to(dtype).contiguous(),
        hit_cov=torch.as_tensor(np.ascontiguousarray(ev.hit_cov), device=dev).to(dtype).contiguous(),
    )


def plane_event_tensors(ev, dtype=torch.float32, device="cuda"):
    """Device copies of a tilted-module batch: hit_offsets [n+1], hit_module
    [n_hits] int32, hit_valid, hit_uv [2][n_hits], hit_cov_uv [3][n_hits]."""
    dev = torch.device(device)
    return dict(
        hit_offsets=torch.as_tensor(np.ascontiguousarray(ev.hit_offsets, np.int32), device=dev),
        hit_module=torch.as_tensor(np.ascontiguousarray(ev.hit_module, np.int32), device=dev),
        hit_valid=torch.as_tensor(np.ascontiguousarray(ev.hit_valid, np.uint8), device=dev),
        hit_uv=torch.as_tensor(np.ascontiguousarray(ev.hit_uv), device=dev).to(dtype).contiguous(),
        hit_cov_uv=torch.as_tensor(np.ascontiguousarray(ev.hit_cov_uv), device=dev).to(dtype).contiguous(),
    )
