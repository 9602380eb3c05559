"""MI355X (gfx950) inverse ray shooting for microlensing magnification maps.

Python binding of the C ABI in include/irs.h (libirs.so, built from csrc/).
Argument marshalling only: every step of the path runs in the HIP kernels.
Device buffers and streams may come from PyTorch tensors; the library itself
does not depend on torch.
"""
import ctypes as C

import numpy as np

from . import _ffi
from ._ffi import (IRS_DIRECT, IRS_INTERP, IRS_LEARNED, IRS_FP64, IRS_FP32_KAHAN, IRS_SHEET_OFF,
                   IRS_OUT_ON_DEVICE, IRS_TIME_PHASES, IRS_LEARN_NFREQ, IRS_LEARN_NPARAMS,
                   IRS_LEARN_FIELDS, EXPORTS, Params, GeometryInfo, MapStats, LearnParams,
                   LearnReport)

__all__ = ["IrsError", "make_params", "params_from_workload", "geometry", "level1_span",
           "source_side_for_n_star", "Plan", "Batch", "load",
           "learn_params", "mlp_forward", "mlp_loss_grad", "IRS_DIRECT", "IRS_INTERP",
           "IRS_LEARNED", "IRS_FP64", "IRS_FP32_KAHAN", "IRS_LEARN_NPARAMS", "IRS_LEARN_FIELDS",
           "EXPORTS"]

load = _ffi.load

_METHODS = {"direct": IRS_DIRECT, "interp": IRS_INTERP, "learned": IRS_LEARNED}
_PRECISIONS = {"fp64": IRS_FP64, "fp32": IRS_FP32_KAHAN, "fp32_kahan": IRS_FP32_KAHAN}


class IrsError(RuntimeError):
    def __init__(self, status, where):
        lib = _ffi.load()
        msg = lib.irs_last_error().decode(errors="replace")
        self.status = status
        super().__init__(f"{where}: {_ffi.STATUS_NAMES.get(status, status)}: {msg}")


def _check(status, where):
    if status != 0:
        raise IrsError(status, where)


def make_params(kappa_star, kappa_c, gamma, source_side, npix, rays_per_pixel=0.0, n_rays=0,
                border=-1.0, method="direct", precision="fp64", level2_spacing=0.0,
                level2_ray_multiple=0.0, crit_eps=0.0, sheet=True,
                level2_paper=False, circle=False) -> Params:
    return Params(float(kappa_star), float(kappa_c), float(gamma), float(source_side),
                  int(npix), float(rays_per_pixel), int(n_rays),
                  float(-1.0 if border is None else border),
                  _METHODS[method] if isinstance(method, str) else int(method),
                  _PRECISIONS[precision] if isinstance(precision, str) else int(precision),
                  float(level2_spacing or 0.0), float(level2_ray_multiple or 0.0),
                  float(crit_eps),
                  (0 if sheet else IRS_SHEET_OFF) | (_ffi.IRS_LEVEL2_PAPER if level2_paper else 0)
                  | (_ffi.IRS_CIRCLE if circle else 0))


def params_from_workload(w, method="direct", precision="fp64", **over) -> Params:
    """Params from any object with the workload fields (kappa_star, kappa_c,
    gamma, source_side, npix, rays_per_pixel, n_rays, level2_ray_multiple)."""
    kw = dict(kappa_star=w.kappa_star, kappa_c=w.kappa_c, gamma=w.gamma,
              source_side=w.source_side, npix=w.npix, rays_per_pixel=w.rays_per_pixel,
              n_rays=w.n_rays, level2_ray_multiple=getattr(w, "level2_ray_multiple", 0.0),
              method=method, precision=precision)
    kw.update(over)
    return make_params(**kw)


def geometry(params: Params, n_lens: int = 0) -> dict:
    """irs_geometry: the plan geometry on the host (no GPU needed)."""
    lib = _ffi.load()
    out = GeometryInfo()
    _check(lib.irs_geometry(C.byref(params), int(n_lens), C.byref(out)), "irs_geometry")
    return out.as_dict()


def source_side_for_n_star(kappa_star, kappa_c, gamma, n_star, **kw) -> float:
    """irs_source_side: the source side S whose rectangle holds n_star lenses
    by the lens-count rule (irs_geometry's n_stars_expected)."""
    lib = _ffi.load()
    s = C.c_double()
    p = make_params(kappa_star, kappa_c, gamma, 1.0, 16, n_rays=1, **kw)
    _check(lib.irs_source_side(C.byref(p), int(n_star), C.byref(s)), "irs_source_side")
    return s.value


def level1_span(geometry_info: dict, axis: int, c: int):
    """irs_level1_span: ray rows (axis 1) or columns (axis 0) [first, last)
    whose level-2 points lie in level-1 row (column) c of a geometry dict."""
    lib = _ffi.load()
    gi = GeometryInfo(**{k: geometry_info[k] for k, _ in GeometryInfo._fields_})
    a, b = C.c_int64(), C.c_int64()
    _check(lib.irs_level1_span(C.byref(gi), int(axis), int(c), C.byref(a), C.byref(b)),
           "irs_level1_span")
    return a.value, b.value


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _vp(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t):
    return C.c_void_p(t.data_ptr())


def learn_params(**over) -> LearnParams:
    """Training settings: the library's defaults with keyword overrides."""
    lib = _ffi.load()
    lp = LearnParams()
    _check(lib.irs_learn_defaults(C.byref(lp)), "irs_learn_defaults")
    for k, v in over.items():
        if not hasattr(lp, k):
            raise KeyError(k)
        setattr(lp, k, v)
    return lp


def _f32(a, n):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != n:
        raise ValueError(f"expected {n} float32 values, got {a.size}")
    return a


def mlp_forward(freqs, theta, h, y, stream=None):
    """Network outputs into y (device tensor, 16 x n float32) for offsets h
    (device tensor, 2 x n float32: hx row, then hy row)."""
    lib = _ffi.load()
    n = h.shape[-1]
    fr, th = _f32(freqs, 2 * IRS_LEARN_NFREQ), _f32(theta, IRS_LEARN_NPARAMS)
    s = None if stream is None else C.c_void_p(int(stream))
    _check(lib.irs_mlp_forward(int(n), _vp(fr), _vp(th), _dev_ptr(h), _dev_ptr(y), s),
           "irs_mlp_forward")


def mlp_loss_grad(freqs, theta, samples, n, stream=None):
    """(loss, gradient float32 [IRS_LEARN_NPARAMS]) of the training kernels over
    n sample records (device tensor, IRS_LEARN_FIELDS x n float32)."""
    lib = _ffi.load()
    fr, th = _f32(freqs, 2 * IRS_LEARN_NFREQ), _f32(theta, IRS_LEARN_NPARAMS)
    g = np.empty(IRS_LEARN_NPARAMS, np.float32)
    loss = C.c_double()
    s = None if stream is None else C.c_void_p(int(stream))
    _check(lib.irs_mlp_loss_grad(int(n), _vp(fr), _vp(th), _dev_ptr(samples), C.byref(loss),
                                 _vp(g), s), "irs_mlp_loss_grad")
    return loss.value, g


class Plan:
    """A plan: geometry + lenses resident on the current HIP device."""

    def __init__(self, params: Params, x, y, m=None, stream=None):
        lib = _ffi.load()
        self._lib = lib
        self.params = params
        x, y, m = _f64(x), _f64(y), _f64(m)
        if x.shape != y.shape or (m is not None and m.shape != x.shape):
            raise ValueError("x, y (and m) must have the same length")
        handle = C.c_void_p()
        s = None if stream is None else C.c_void_p(int(stream))
        _check(lib.irs_plan(C.byref(params), int(x.size), _vp(x), _vp(y), _vp(m), s,
                            C.byref(handle)), "irs_plan")
        self._h = handle
        gi = GeometryInfo()
        _check(lib.irs_plan_geometry(self._h, C.byref(gi)), "irs_plan_geometry")
        self.geometry = gi.as_dict()

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.irs_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def n_rays(self) -> int:
        return self.geometry["nx"] * self.geometry["ny"]

    def level1(self):
        """The level-1 packing: (cell_start[n1x*n1y + 1], order[n_lens]) as int32
        host arrays; packed lens k is input lens order[k]."""
        g = self.geometry
        cs = np.empty(g["n1x"] * g["n1y"] + 1, np.int32)
        order = np.empty(max(g["n_lens"], 1), np.int32)
        _check(self._lib.irs_plan_level1(self._h, _vp(cs), _vp(order)), "irs_plan_level1")
        return cs, order[:g["n_lens"]]

    def deflect_grid(self, first_ray: int, n: int, alpha=True, pixel=True):
        """Per-ray alpha1, alpha2 (FP64) and pixel index (-1 off map), host arrays."""
        a1 = np.empty(n) if alpha else None
        a2 = np.empty(n) if alpha else None
        px = np.empty(n, np.int64) if pixel else None
        _check(self._lib.irs_deflect_grid(self._h, int(first_ray), int(n), _vp(a1), _vp(a2),
                                          _vp(px), 0), "irs_deflect_grid")
        return a1, a2, px

    def deflect_grid_device(self, first_ray: int, n: int, a1, a2, px):
        """Same as deflect_grid into caller-owned device tensors (any may be None)."""
        _check(self._lib.irs_deflect_grid(self._h, int(first_ray), int(n),
                                          None if a1 is None else _dev_ptr(a1),
                                          None if a2 is None else _dev_ptr(a2),
                                          None if px is None else _dev_ptr(px),
                                          IRS_OUT_ON_DEVICE), "irs_deflect_grid")

    def shoot_map(self, time_phases=False):
        """Full map on the host: (counts uint32 [npix, npix], stats dict)."""
        npix = self.params.npix_side
        counts = np.zeros(npix * npix, np.uint32)
        st = MapStats()
        fl = IRS_TIME_PHASES if time_phases else 0
        _check(self._lib.irs_shoot_map(self._h, _vp(counts), C.byref(st), fl), "irs_shoot_map")
        return counts.reshape(npix, npix), st.as_dict()

    def shoot_map_device(self, counts, time_phases=False):
        """Full map into a device tensor of npix^2 32-bit integers (overwritten).
        Returns the stats dict."""
        st = MapStats()
        fl = IRS_OUT_ON_DEVICE | (IRS_TIME_PHASES if time_phases else 0)
        _check(self._lib.irs_shoot_map(self._h, _dev_ptr(counts), C.byref(st), fl), "irs_shoot_map")
        return st.as_dict()

    def shoot_rows(self, row0: int, nrows: int, counts, time_phases=False):
        """Add rows [row0, row0+nrows) into counts: a host uint32 array or a
        device tensor of npix^2 32-bit integers.  Returns the stats dict."""
        st = MapStats()
        fl = IRS_TIME_PHASES if time_phases else 0
        if isinstance(counts, np.ndarray):
            if counts.dtype != np.uint32 or not counts.flags.c_contiguous:
                raise ValueError("host counts must be a contiguous uint32 array")
            _check(self._lib.irs_shoot_rows(self._h, int(row0), int(nrows), _vp(counts),
                                            C.byref(st), fl), "irs_shoot_rows")
        else:
            _check(self._lib.irs_shoot_rows(self._h, int(row0), int(nrows), _dev_ptr(counts),
                                            C.byref(st), fl | IRS_OUT_ON_DEVICE),
                   "irs_shoot_rows")
        return st.as_dict()

    def shoot_rows_noalloc(self, row0: int, nrows: int, counts, want_landed=True):
        """irs_shoot_rows_noalloc: add rows [row0, row0+nrows) into a device
        tensor of npix^2 32-bit integers without allocating device memory.
        Returns the rays binned (None when want_landed is False: no sync)."""
        n = C.c_int64()
        _check(self._lib.irs_shoot_rows_noalloc(self._h, int(row0), int(nrows), _dev_ptr(counts),
                                                C.byref(n) if want_landed else None),
               "irs_shoot_rows_noalloc")
        return n.value if want_landed else None

    # ---- learned interpolant (method "learned")
    def learn(self, freqs, lp: LearnParams = None, theta0=None) -> dict:
        """Train and validate the network (irs_learn); returns the report."""
        lp = lp if lp is not None else learn_params()
        fr = _f32(freqs, 2 * IRS_LEARN_NFREQ)
        th = None if theta0 is None else _f32(theta0, IRS_LEARN_NPARAMS)
        rep = LearnReport()
        _check(self._lib.irs_learn(self._h, C.byref(lp), _vp(fr), _vp(th), C.byref(rep)),
               "irs_learn")
        return rep.as_dict()

    def learn_set(self, freqs, theta, lp: LearnParams = None) -> dict:
        """Install a network and validate it (irs_learn_set); returns the report."""
        lp = lp if lp is not None else learn_params()
        fr, th = _f32(freqs, 2 * IRS_LEARN_NFREQ), _f32(theta, IRS_LEARN_NPARAMS)
        rep = LearnReport()
        _check(self._lib.irs_learn_set(self._h, C.byref(lp), _vp(fr), _vp(th), C.byref(rep)),
               "irs_learn_set")
        return rep.as_dict()

    def learn_get(self):
        """(frequencies (64, 2), parameters, coarse) of the plan's network."""
        fr = np.empty(2 * IRS_LEARN_NFREQ, np.float32)
        th = np.empty(IRS_LEARN_NPARAMS, np.float32)
        qc = C.c_int32()
        _check(self._lib.irs_learn_get(self._h, _vp(fr), _vp(th), C.byref(qc)), "irs_learn_get")
        return fr.reshape(IRS_LEARN_NFREQ, 2), th, qc.value

    def learn_corners(self, coarse: int, row0: int, nrows: int) -> np.ndarray:
        """Corner table of level-1 rows [row0, row0+nrows): complex (A, A') arrays
        shaped (nrows, n1x, coarse+1, coarse+1)."""
        g = self.geometry
        q1 = coarse + 1
        out = np.empty(nrows * g["n1x"] * q1 * q1 * 4)
        _check(self._lib.irs_learn_corners(self._h, int(coarse), int(row0), int(nrows), _vp(out)),
               "irs_learn_corners")
        o = out.reshape(nrows, g["n1x"], q1, q1, 4)
        return o[..., 0] + 1j * o[..., 1], o[..., 2] + 1j * o[..., 3]

    def learn_samples(self, coarse: int, row0: int, nrows: int, per_cell: int, seed: int, out):
        """Exact samples into a device tensor of IRS_LEARN_FIELDS x n float32,
        n = nrows * n1x * per_cell."""
        _check(self._lib.irs_learn_samples(self._h, int(coarse), int(row0), int(nrows),
                                           int(per_cell), int(seed), _dev_ptr(out)),
               "irs_learn_samples")

    def learn_weights(self, h, y):
        """The plan's learned weights, as its rays take them, into y (device
        tensor, 16 x n float32) at offsets h (device tensor, 2 x n float32)."""
        _check(self._lib.irs_learn_weights(self._h, int(h.shape[-1]), _dev_ptr(h), _dev_ptr(y)),
               "irs_learn_weights")

    def set_direct_variant(self, v: int):
        """FP32 direct tile shape (0, 1, 2); results are identical for all."""
        _check(self._lib.irs_plan_set_direct_variant(self._h, int(v)),
               "irs_plan_set_direct_variant")

    def level1_row_rays(self, c: int):
        """Ray rows [j0, j1) whose level-2 points lie in level-1 row c."""
        return level1_span(self.geometry, 1, c)

    def level1_col_rays(self, c: int):
        """Ray columns [i0, i1) whose level-2 points lie in level-1 column c."""
        return level1_span(self.geometry, 0, c)


class Batch:
    """Independent maps run together in one graph launch (see irs_batch_run)."""

    def __init__(self, plans, stream=None):
        lib = _ffi.load()
        self._lib = lib
        self.plans = list(plans)
        arr = (C.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = C.c_void_p()
        s = None if stream is None else C.c_void_p(int(stream))
        _check(lib.irs_batch_create(arr, len(self.plans), s, C.byref(h)), "irs_batch_create")
        self._h = h

    def tune(self, cache_path=None):
        _check(self._lib.irs_batch_tune(self._h, None if cache_path is None
                                        else str(cache_path).encode()), "irs_batch_tune")
        return self.info()

    def info(self) -> dict:
        out = _ffi.BatchInfo()
        _check(self._lib.irs_batch_get_info(self._h, C.byref(out)), "irs_batch_get_info")
        return out.as_dict()

    def run(self, counts):
        """counts: one device tensor (npix^2 32-bit ints) per plan, overwritten."""
        ptrs = (C.c_void_p * len(counts))(*[t.data_ptr() for t in counts])
        st = (MapStats * len(counts))()
        _check(self._lib.irs_batch_run(self._h, ptrs, st, 0), "irs_batch_run")
        return [s.as_dict() for s in st]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.irs_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
