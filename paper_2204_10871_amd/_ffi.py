"""ctypes declarations of the C ABI in include/irs.h (marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libirs.so")

IRS_OK, IRS_E_INVALID, IRS_E_CRITICAL, IRS_E_NOMEM, IRS_E_DEVICE, IRS_E_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "IRS_OK", 1: "IRS_E_INVALID", 2: "IRS_E_CRITICAL", 3: "IRS_E_NOMEM",
                4: "IRS_E_DEVICE", 5: "IRS_E_UNSUPPORTED"}
IRS_DIRECT, IRS_INTERP, IRS_LEARNED = 0, 1, 2
IRS_FP64, IRS_FP32_KAHAN = 0, 1
IRS_SHEET_OFF = 1 << 0
IRS_LEVEL2_PAPER = 1 << 1
IRS_CIRCLE = 1 << 2
IRS_OUT_ON_DEVICE = 1 << 8
IRS_TIME_PHASES = 1 << 9
IRS_LEARN_NFREQ = 64
IRS_LEARN_NPARAMS = 68112
IRS_LEARN_FIELDS = 24

# every function include/irs.h declares
EXPORTS = ("irs_geometry", "irs_level1_span", "irs_source_side", "irs_plan", "irs_deflect_grid",
           "irs_shoot_rows", "irs_shoot_rows_noalloc", "irs_shoot_map",
           "irs_plan_set_direct_variant", "irs_plan_geometry", "irs_plan_level1", "irs_free",
           "irs_last_error", "irs_debug_fail_alloc", "irs_debug_live_allocs",
           "irs_batch_create", "irs_batch_tune", "irs_batch_run", "irs_batch_get_info",
           "irs_batch_free", "irs_learn_defaults", "irs_learn", "irs_learn_set", "irs_learn_get",
           "irs_learn_corners", "irs_learn_samples", "irs_learn_weights", "irs_mlp_forward",
           "irs_mlp_loss_grad")


class Params(C.Structure):
    _fields_ = [("kappa_star", C.c_double), ("kappa_c", C.c_double), ("gamma", C.c_double),
                ("source_side", C.c_double), ("npix_side", C.c_int64),
                ("rays_per_pixel", C.c_double), ("n_rays", C.c_int64), ("border", C.c_double),
                ("method", C.c_int32), ("precision", C.c_int32),
                ("level2_spacing", C.c_double), ("level2_ray_multiple", C.c_double),
                ("crit_eps", C.c_double), ("flags", C.c_uint64)]


class GeometryInfo(C.Structure):
    _fields_ = [("kappa", C.c_double), ("border", C.c_double), ("ix", C.c_double),
                ("iy", C.c_double), ("a1", C.c_double), ("a2", C.c_double), ("b1", C.c_double),
                ("b2", C.c_double), ("n_rays_target", C.c_int64), ("dx3", C.c_double),
                ("nx", C.c_int64), ("ny", C.c_int64), ("ray_dx", C.c_double),
                ("ray_dy", C.c_double), ("n_lens", C.c_int64), ("dx1", C.c_double),
                ("n1x", C.c_int64), ("n1y", C.c_int64), ("dx2", C.c_double), ("q", C.c_int64),
                ("dpix", C.c_double), ("s_img", C.c_double), ("s_src", C.c_double),
                ("mu_th", C.c_double), ("n_stars_expected", C.c_int64),
                ("lens_radius", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class MapStats(C.Structure):
    _fields_ = [("rays_shot", C.c_int64), ("rays_landed", C.c_int64), ("rays_off", C.c_int64),
                ("n_lens", C.c_int64), ("kappa_star_eff", C.c_double), ("ms_total", C.c_double),
                ("level2_points", C.c_int64), ("level2_pairs", C.c_int64),
                ("direct_pairs", C.c_int64), ("level2_flops", C.c_double),
                ("level2_expand_flops", C.c_double),
                ("n_level2_launches", C.c_int32),
                ("n_ray_launches", C.c_int32), ("ms_level2", C.c_double),
                ("ms_level2_expand", C.c_double), ("ms_rays", C.c_double),
                ("learned", C.c_int32), ("pad_", C.c_int32), ("ray_flops", C.c_double),
                ("super_cells", C.c_int32), ("mid_cells", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class BatchInfo(C.Structure):
    _fields_ = [("n_maps", C.c_int32), ("method", C.c_int32), ("precision", C.c_int32),
                ("direct_variant", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("band_rows", C.c_int32), ("tuned", C.c_int32), ("from_cache", C.c_int32),
                ("work_items", C.c_int64), ("tune_ms", C.c_double), ("whole_maps", C.c_int32),
                ("maps_per_launch", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class LearnParams(C.Structure):
    _fields_ = [("coarse", C.c_int32), ("train_rows", C.c_int32), ("n_samples", C.c_int64),
                ("n_val", C.c_int64), ("batch", C.c_int32), ("steps", C.c_int32),
                ("lr", C.c_float), ("lr_final", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("adam_eps", C.c_float), ("pad_", C.c_int32),
                ("seed", C.c_uint64), ("tol_mean", C.c_double), ("tol_p9999", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad_"}


class LearnReport(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("n_val", C.c_int64), ("steps", C.c_int64),
                ("loss_first", C.c_double), ("loss_last", C.c_double),
                ("val_mean_abs", C.c_double), ("val_p9999_abs", C.c_double),
                ("val_max_abs", C.c_double), ("base_mean_abs", C.c_double),
                ("base_p9999_abs", C.c_double), ("base_max_abs", C.c_double),
                ("tol_mean", C.c_double), ("tol_p9999", C.c_double), ("fallback", C.c_int32),
                ("coarse", C.c_int32), ("ms_samples", C.c_double), ("ms_train", C.c_double),
                ("ms_validate", C.c_double), ("corner_bytes_per_row", C.c_int64),
                ("coef_bytes_per_row", C.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load():
    """Load libirs.so, failing loudly when it has not been built.

    PyTorch wheels bundle their own HIP runtime under the same soname as
    ROCm's (libamdhip64.so.7).  When PyTorch is installed it is imported
    first, so the library binds to that runtime and both share one HIP
    runtime (device pointers and streams can then be passed between them).
    """
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401  (see docstring)
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it first "
                           "(python -m paper_2204_10871_amd.build or __graft_entry__.build())")
    _lib = declare(C.CDLL(LIB_PATH))
    return _lib


def declare(lib):
    """Argument and result types of every entry point on a loaded copy of
    the library; returns lib."""
    P, vp, i64, u64 = C.POINTER, C.c_void_p, C.c_int64, C.c_uint64
    lib.irs_geometry.argtypes = [P(Params), i64, P(GeometryInfo)]
    lib.irs_level1_span.argtypes = [P(GeometryInfo), C.c_int32, i64, P(i64), P(i64)]
    lib.irs_source_side.argtypes = [P(Params), i64, P(C.c_double)]
    lib.irs_plan.argtypes = [P(Params), i64, vp, vp, vp, vp, P(vp)]
    lib.irs_deflect_grid.argtypes = [vp, i64, i64, vp, vp, vp, u64]
    lib.irs_shoot_rows.argtypes = [vp, i64, i64, vp, P(MapStats), u64]
    lib.irs_shoot_rows_noalloc.argtypes = [vp, i64, i64, vp, P(i64)]
    lib.irs_shoot_map.argtypes = [vp, vp, P(MapStats), u64]
    lib.irs_plan_geometry.argtypes = [vp, P(GeometryInfo)]
    lib.irs_plan_level1.argtypes = [vp, vp, vp]
    lib.irs_plan_set_direct_variant.argtypes = [vp, C.c_int32]
    lib.irs_batch_create.argtypes = [P(vp), C.c_int32, vp, P(vp)]
    lib.irs_batch_tune.argtypes = [vp, C.c_char_p]
    lib.irs_batch_run.argtypes = [vp, P(vp), P(MapStats), u64]
    lib.irs_batch_get_info.argtypes = [vp, P(BatchInfo)]
    lib.irs_batch_free.argtypes = [vp]
    lib.irs_batch_free.restype = None
    i32 = C.c_int32
    lib.irs_learn_defaults.argtypes = [P(LearnParams)]
    lib.irs_learn.argtypes = [vp, P(LearnParams), vp, vp, P(LearnReport)]
    lib.irs_learn_set.argtypes = [vp, P(LearnParams), vp, vp, P(LearnReport)]
    lib.irs_learn_get.argtypes = [vp, vp, vp, P(i32)]
    lib.irs_learn_corners.argtypes = [vp, i32, i64, i64, vp]
    lib.irs_learn_samples.argtypes = [vp, i32, i64, i64, i32, u64, vp]
    lib.irs_learn_weights.argtypes = [vp, i64, vp, vp]
    lib.irs_mlp_forward.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.irs_mlp_loss_grad.argtypes = [i64, vp, vp, vp, P(C.c_double), vp, vp]
    lib.irs_free.argtypes = [vp]
    lib.irs_free.restype = None
    lib.irs_debug_fail_alloc.argtypes = [i64]
    lib.irs_debug_fail_alloc.restype = C.c_int
    lib.irs_debug_live_allocs.argtypes = [vp, vp]
    lib.irs_debug_live_allocs.restype = C.c_int
    lib.irs_last_error.argtypes = []
    lib.irs_last_error.restype = C.c_char_p
    for name in ("irs_geometry", "irs_level1_span", "irs_source_side", "irs_plan",
                 "irs_deflect_grid", "irs_shoot_rows", "irs_shoot_rows_noalloc", "irs_shoot_map",
                 "irs_plan_geometry", "irs_plan_level1", "irs_plan_set_direct_variant",
                 "irs_batch_create", "irs_batch_tune", "irs_batch_run", "irs_batch_get_info",
                 "irs_learn_defaults", "irs_learn", "irs_learn_set", "irs_learn_get",
                 "irs_learn_corners", "irs_learn_samples", "irs_learn_weights",
                 "irs_mlp_forward", "irs_mlp_loss_grad"):
        getattr(lib, name).restype = C.c_int
    return lib
