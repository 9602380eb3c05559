"""Calls of the C ABI that need no GPU, with their results, to compare two
builds of the library (the sanitizer build against the regular one): the
geometry of valid and invalid parameter sets, level-1 spans, the source side
for a lens count, the learning defaults, every entry point's NULL and
out-of-range arguments, and plan set-up up to the first device call."""
import ctypes as C

import numpy as np

import paper_2204_10871_amd as irs
from paper_2204_10871_amd import _ffi

_VALID = [
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=256, n_rays=2048 ** 2),
    dict(kappa_star=0.45, kappa_c=0.05, gamma=0.45, source_side=25.0, npix=4096,
         rays_per_pixel=100.0, level2_ray_multiple=16.0, method="interp"),
    dict(kappa_star=0.6, kappa_c=0.0, gamma=0.6, source_side=1007.8, npix=10000,
         rays_per_pixel=1000.0, method="interp"),
    dict(kappa_star=0.0, kappa_c=0.23, gamma=0.11, source_side=3.7, npix=37, n_rays=611 * 577,
         border=0.37),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=64, rays_per_pixel=10.0,
         circle=True),
    dict(kappa_star=0.5, kappa_c=0.05, gamma=0.5, source_side=30.0, npix=512,
         rays_per_pixel=4.0, method="learned"),
    dict(kappa_star=0.2, kappa_c=0.2, gamma=0.1, source_side=5.0, npix=1, n_rays=1,
         method="interp", precision="fp64"),
]
_INVALID = [
    dict(kappa_star=0.5, kappa_c=0.0, gamma=0.5, source_side=100.0, npix=64, rays_per_pixel=10.0),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=0, rays_per_pixel=10.0),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=46341,
         rays_per_pixel=1.0),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=-1.0, npix=64, rays_per_pixel=10.0),
    dict(kappa_star=float("nan"), kappa_c=0.0, gamma=0.3, source_side=10.0, npix=64,
         rays_per_pixel=10.0),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=float("inf"), source_side=10.0, npix=64,
         rays_per_pixel=10.0),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=64, rays_per_pixel=0.0),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=64, rays_per_pixel=10.0,
         circle=True, method="interp"),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=64, rays_per_pixel=10.0,
         method="interp", level2_spacing=1e-6),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=1e30, npix=64, rays_per_pixel=10.0,
         method="interp"),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=1e9, npix=64, n_rays=1 << 62),
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=64, rays_per_pixel=10.0,
         method=7),
]
_LENS_COUNTS = [0, 1, 105, 100000, -1, 1 << 40]


def _fields(s):
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        out[name] = v.hex() if isinstance(v, float) else v
    return out


def _error(lib):
    return lib.irs_last_error().decode(errors="replace")


def run(path):
    lib = _ffi.declare(C.CDLL(path))
    out = {}
    for i, kw in enumerate(_VALID + _INVALID):
        p = irs.make_params(**kw)
        for n in _LENS_COUNTS:
            gi = _ffi.GeometryInfo()
            st = lib.irs_geometry(C.byref(p), n, C.byref(gi))
            out[f"geometry {i} {n}"] = [st, _fields(gi) if st == 0 else _error(lib)]
            if st != 0 or n != 100000:
                continue
            spans = []
            for axis, ncell in ((0, gi.n1x), (1, gi.n1y)):
                for c in sorted(set(list(range(min(ncell, 40))) + [ncell - 1, ncell, -1])):
                    a, b = C.c_int64(-7), C.c_int64(-7)
                    s = lib.irs_level1_span(C.byref(gi), axis, c, C.byref(a), C.byref(b))
                    spans.append([axis, c, s, a.value, b.value])
            a, b = C.c_int64(), C.c_int64()
            spans.append([2, 0, lib.irs_level1_span(C.byref(gi), 2, 0, C.byref(a), C.byref(b))])
            out[f"spans {i}"] = spans
        side = C.c_double(-1.0)
        for n in (1, 1000, 1000000, 0, -5):
            s = lib.irs_source_side(C.byref(p), n, C.byref(side))
            out[f"side {i} {n}"] = [s, side.value.hex() if s == 0 else _error(lib)]
    lp = _ffi.LearnParams()
    out["learn defaults"] = [lib.irs_learn_defaults(C.byref(lp)), _fields(lp)]

    # NULL and out-of-range arguments: refused before any device call
    calls = {
        "geometry": lambda: lib.irs_geometry(None, 0, None),
        "level1_span": lambda: lib.irs_level1_span(None, 0, 0, None, None),
        "source_side": lambda: lib.irs_source_side(None, 10, None),
        "plan": lambda: lib.irs_plan(None, 0, None, None, None, None, None),
        "deflect_grid": lambda: lib.irs_deflect_grid(None, 0, 1, None, None, None, 0),
        "shoot_rows": lambda: lib.irs_shoot_rows(None, 0, 1, None, None, 0),
        "shoot_rows_noalloc": lambda: lib.irs_shoot_rows_noalloc(None, 0, 1, None, None),
        "shoot_map": lambda: lib.irs_shoot_map(None, None, None, 0),
        "plan_geometry": lambda: lib.irs_plan_geometry(None, None),
        "plan_level1": lambda: lib.irs_plan_level1(None, None, None),
        "set_direct_variant": lambda: lib.irs_plan_set_direct_variant(None, 1),
        "batch_create": lambda: lib.irs_batch_create(None, 0, None, None),
        "batch_tune": lambda: lib.irs_batch_tune(None, None),
        "batch_run": lambda: lib.irs_batch_run(None, None, None, 0),
        "batch_info": lambda: lib.irs_batch_get_info(None, None),
        "learn_defaults": lambda: lib.irs_learn_defaults(None),
        "learn": lambda: lib.irs_learn(None, None, None, None, None),
        "learn_set": lambda: lib.irs_learn_set(None, None, None, None, None),
        "learn_get": lambda: lib.irs_learn_get(None, None, None, None),
        "learn_corners": lambda: lib.irs_learn_corners(None, 8, 0, 1, None),
        "learn_samples": lambda: lib.irs_learn_samples(None, 8, 0, 1, 4, 1, None),
        "learn_weights": lambda: lib.irs_learn_weights(None, 4, None, None),
        "learn_weights": lambda: lib.irs_learn_weights(None, 4, None, None),
        "mlp_forward": lambda: lib.irs_mlp_forward(-1, None, None, None, None, None),
        "mlp_loss_grad": lambda: lib.irs_mlp_loss_grad(-1, None, None, None, None, None, None),
        "fail_alloc": lambda: lib.irs_debug_fail_alloc(-1),
        "live_allocs": lambda: lib.irs_debug_live_allocs(None, None),
    }
    for name, f in calls.items():
        out[f"call {name}"] = [f(), _error(lib)]
    lib.irs_free(None)
    lib.irs_batch_free(None)

    # plan set-up: the host checks of the lenses, then (no GPU here) the
    # first device call's error
    rng = np.random.default_rng(5)
    for i, kw in enumerate(_VALID[:3]):
        p = irs.make_params(**kw)
        gi = _ffi.GeometryInfo()
        lib.irs_geometry(C.byref(p), 500, C.byref(gi))
        x = rng.uniform(gi.a1, gi.a2, 500)
        y = rng.uniform(gi.b1, gi.b2, 500)
        m = rng.uniform(0.1, 1.0, 500)
        bad = x.copy()
        bad[17] = np.nan
        far = x.copy()
        far[3] = gi.a2 + 10.0
        for tag, xx, mm in (("ok", x, None), ("masses", x, m), ("nan", bad, None),
                            ("outside", far, None), ("negative mass", x, -m)):
            h = C.c_void_p()
            st = lib.irs_plan(C.byref(p), 500, xx.ctypes.data, y.ctypes.data,
                              None if mm is None else mm.ctypes.data, None, C.byref(h))
            out[f"plan {i} {tag}"] = [st, h.value is None]
            if h.value is not None:
                lib.irs_free(h)
        h = C.c_void_p()
        out[f"plan {i} null x"] = [lib.irs_plan(C.byref(p), 500, None, y.ctypes.data, None,
                                                None, C.byref(h)), h.value is None]
    return out
