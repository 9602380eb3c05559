"""ctypes front end of the C oracle (irs_oracle.c).  Test infrastructure only.

Argument marshalling and the build step live here; all arithmetic of O-1 and
O-2 is in irs_oracle.c.  The shared object is compiled with gcc from the
committed source (plain -O2, no FMA contraction, portable x86-64).
"""
import ctypes as C
import os
import subprocess
import threading

import numpy as np

from .geometry import Geometry

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "irs_oracle.c")
# IRS_ORACLE_LIB: load a prebuilt copy instead (the sanitizer build of the tests)
_LIB_ENV = os.environ.get("IRS_ORACLE_LIB", "")
_LIB = _LIB_ENV or os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


class _Setup(C.Structure):
    _fields_ = [("kappa_star", C.c_double), ("kappa", C.c_double), ("gamma", C.c_double),
                ("a1", C.c_double), ("a2", C.c_double), ("b1", C.c_double), ("b2", C.c_double),
                ("nx", C.c_int64), ("ny", C.c_int64), ("source_side", C.c_double),
                ("npix", C.c_int64), ("sheet", C.c_int64), ("n1x", C.c_int64),
                ("n1y", C.c_int64), ("q", C.c_int64)]


def build(force: bool = True) -> str:
    """Compile irs_oracle.c into liboracle.so (gcc, OpenMP)."""
    lib = os.path.join(_HERE, "liboracle.so")
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build_sanitized(path: str) -> str:
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal) into path, for IRS_ORACLE_LIB.  A process that loads
    it must preload gcc's libasan and libubsan."""
    cmd = ["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-o", path, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return path


def load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not _LIB_ENV and ((not os.path.exists(_LIB)) or
                             os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER
        d, i64, vp = C.c_double, C.c_int64, C.c_void_p
        lib.orc_sheet_I.argtypes = [d, d, d, d, i64, vp, vp, vp, vp]
        lib.orc_alpha_points.argtypes = [P(_Setup), i64, vp, vp, vp, i64, vp, vp, vp, vp, vp]
        lib.orc_shoot_direct.argtypes = [P(_Setup), i64, vp, vp, vp, i64, i64, vp, vp, vp,
                                         vp, vp, vp, C.c_int]
        lib.orc_level1.argtypes = [P(_Setup), i64, vp, vp, vp, vp]
        lib.orc_level2.argtypes = [P(_Setup), i64, vp, vp, vp, vp, vp, i64, vp, vp, vp, C.c_int]
        lib.orc_shoot_interp.argtypes = [P(_Setup), i64, vp, vp, vp, vp, vp, vp, i64, i64, vp,
                                         vp, vp, vp, vp, vp, C.c_int]
        lib.orc_shoot_interp_rays.argtypes = [P(_Setup), i64, vp, vp, vp, vp, vp, i64, i64, vp,
                                              vp, vp, vp, vp, vp, C.c_int]
        lib.orc_sheet_taylor_xy.argtypes = [P(_Setup), d, d, vp]
        lib.orc_far_point.argtypes = [P(_Setup), i64, vp, vp, vp, vp, vp, i64, vp, vp, vp, vp,
                                      vp, C.c_int]
        _lib = lib
        return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def setup_of(g: Geometry) -> _Setup:
    return _Setup(g.kappa_star, g.kappa, g.gamma, g.a1, g.a2, g.b1, g.b2, g.nx, g.ny,
                  g.source_side, g.npix, (2 if g.circle else 1) if g.sheet else 0, g.n1x,
                  g.n1y, g.q)


def sheet_I(rect, x, y):
    """Appendix A closed forms with A = 1 at points (x, y): returns (I1, I2).
    Pinned by 2-D quadrature of the defining integral, div = 2 pi, curl = 0,
    symmetric-square and long-strip limits (tests/test_oracle_sheet.py)."""
    lib = load()
    x, y = _f64(np.atleast_1d(x)), _f64(np.atleast_1d(y))
    I1, I2 = np.empty_like(x), np.empty_like(x)
    a1, a2, b1, b2 = rect
    lib.orc_sheet_I(a1, a2, b1, b2, x.size, _ptr(x), _ptr(y), _ptr(I1), _ptr(I2))
    return I1, I2


def alpha_points(g: Geometry, lenses, x, y):
    """Eq. 6 at arbitrary points.  Returns (alpha1, alpha2, n_singular).
    Pinned by the point-lens magnification, the star-free exact map, the map
    mean vs mu_th and 50-digit brute force (tests/test_oracle_*.py)."""
    lib = load()
    s = setup_of(g)
    x, y = _f64(np.atleast_1d(x)), _f64(np.atleast_1d(y))
    ax, ay = np.empty_like(x), np.empty_like(x)
    ns = np.zeros(1, np.int64)
    lx, ly, lm = _f64(lenses.x), _f64(lenses.y), _f64(lenses.m)
    lib.orc_alpha_points(C.byref(s), lenses.n, _ptr(lx), _ptr(ly), _ptr(lm), x.size,
                         _ptr(x), _ptr(y), _ptr(ax), _ptr(ay), _ptr(ns))
    return ax, ay, int(ns[0])


def shoot_direct(g: Geometry, lenses, first=0, n=None, ray_ids=None, want_alpha=True,
                 want_pix=True, want_counts=True, threads=0):
    """O-1 over a ray range or an explicit list of ray ids.

    Returns dict(alpha1, alpha2, pix, counts (npix*npix uint32), landed, off,
    singular).  Pinned as alpha_points, plus ray-count conservation."""
    lib = load()
    s = setup_of(g)
    if ray_ids is not None:
        ray_ids = np.ascontiguousarray(ray_ids, dtype=np.int64)
        n = ray_ids.size
    elif n is None:
        n = g.n_rays - first
    ax = np.empty(n) if want_alpha else None
    ay = np.empty(n) if want_alpha else None
    pix = np.empty(n, np.int64) if want_pix else None
    counts = np.zeros(g.npix * g.npix, np.uint32) if want_counts else None
    st = np.zeros(3, np.int64)
    lx, ly, lm = _f64(lenses.x), _f64(lenses.y), _f64(lenses.m)
    lib.orc_shoot_direct(C.byref(s), lenses.n, _ptr(lx), _ptr(ly), _ptr(lm), first, n,
                         _ptr(ray_ids), _ptr(ax), _ptr(ay), _ptr(pix), _ptr(counts),
                         _ptr(st), threads)
    return dict(alpha1=ax, alpha2=ay, pix=pix, counts=counts, landed=int(st[0]),
                off=int(st[1]), singular=int(st[2]))


def level1(g: Geometry, lenses):
    """Level-1 packing (stable counting sort by cell).  Returns (cell_start, perm).
    Pinned by the partition property (every lens in exactly one cell, cells
    hold exactly the lenses whose positions fall in them)."""
    lib = load()
    s = setup_of(g)
    cs = np.empty(g.n1x * g.n1y + 1, np.int64)
    perm = np.empty(max(lenses.n, 1), np.int64)
    lx, ly = _f64(lenses.x), _f64(lenses.y)
    lib.orc_level1(C.byref(s), lenses.n, _ptr(lx), _ptr(ly), _ptr(cs), _ptr(perm))
    return cs, perm[:lenses.n]


def level2(g: Geometry, lenses, cell_start, perm, gx, gy, threads=0):
    """C_0..C_4 at level-2 points (gx, gy).  Returns complex array (npts, 5).
    Pinned by the exact Taylor remainder identity, h = 0 agreement with O-1,
    the 5th-order convergence of the sheet series and 50-digit brute force."""
    lib = load()
    s = setup_of(g)
    gx = np.ascontiguousarray(np.atleast_1d(gx), np.int64)
    gy = np.ascontiguousarray(np.atleast_1d(gy), np.int64)
    out = np.empty((gx.size, 10))
    lx, ly, lm = _f64(lenses.x), _f64(lenses.y), _f64(lenses.m)
    cs = np.ascontiguousarray(cell_start, np.int64)
    pm = np.ascontiguousarray(perm, np.int64)
    lib.orc_level2(C.byref(s), lenses.n, _ptr(lx), _ptr(ly), _ptr(lm), _ptr(cs), _ptr(pm),
                   gx.size, _ptr(gx), _ptr(gy), _ptr(out), threads)
    return out[:, 0::2] + 1j * out[:, 1::2]


def level2_grid(g: Geometry, lenses, cell_start, perm, threads=0):
    """Coefficients of every level-2 point, row-major (gy, gx): (ny2*nx2, 5) complex."""
    nx2, ny2 = g.n1x * g.q, g.n1y * g.q
    gy, gx = np.meshgrid(np.arange(ny2), np.arange(nx2), indexing="ij")
    return level2(g, lenses, cell_start, perm, gx.ravel(), gy.ravel(), threads)


def shoot_interp(g: Geometry, lenses, cell_start, perm, coef, first=0, n=None,
                 ray_ids=None, want_alpha=True, want_pix=True, want_counts=True, threads=0):
    """O-2 level-3 evaluation with the whole level-2 grid's coefficients `coef`
    (from level2_grid).  Same outputs as shoot_direct."""
    lib = load()
    s = setup_of(g)
    if ray_ids is not None:
        ray_ids = np.ascontiguousarray(ray_ids, dtype=np.int64)
        n = ray_ids.size
    elif n is None:
        n = g.n_rays - first
    cf = np.empty((coef.shape[0], 10))
    cf[:, 0::2], cf[:, 1::2] = coef.real, coef.imag
    ax = np.empty(n) if want_alpha else None
    ay = np.empty(n) if want_alpha else None
    pix = np.empty(n, np.int64) if want_pix else None
    counts = np.zeros(g.npix * g.npix, np.uint32) if want_counts else None
    st = np.zeros(3, np.int64)
    lx, ly, lm = _f64(lenses.x), _f64(lenses.y), _f64(lenses.m)
    cs = np.ascontiguousarray(cell_start, np.int64)
    pm = np.ascontiguousarray(perm, np.int64)
    lib.orc_shoot_interp(C.byref(s), lenses.n, _ptr(lx), _ptr(ly), _ptr(lm), _ptr(cs),
                         _ptr(pm), _ptr(cf), first, n, _ptr(ray_ids), _ptr(ax), _ptr(ay),
                         _ptr(pix), _ptr(counts), _ptr(st), threads)
    return dict(alpha1=ax, alpha2=ay, pix=pix, counts=counts, landed=int(st[0]),
                off=int(st[1]), singular=int(st[2]))


def shoot_interp_rays(g: Geometry, lenses, cell_start, perm, first=0, n=None, ray_ids=None,
                      want_alpha=True, want_pix=True, want_counts=False, threads=0):
    """O-2 for a ray range or list, each ray with the coefficients of its own
    level-2 point summed on the spot (orc_shoot_interp_rays): the same results
    as shoot_interp with the whole level-2 grid (pinned bit for bit against it
    in tests/test_oracle_interp.py) without building that grid, so rays of
    full-size maps can be checked.  Same outputs as shoot_direct."""
    lib = load()
    s = setup_of(g)
    if ray_ids is not None:
        ray_ids = np.ascontiguousarray(ray_ids, dtype=np.int64)
        n = ray_ids.size
    elif n is None:
        n = g.n_rays - first
    ax = np.empty(n) if want_alpha else None
    ay = np.empty(n) if want_alpha else None
    pix = np.empty(n, np.int64) if want_pix else None
    counts = np.zeros(g.npix * g.npix, np.uint32) if want_counts else None
    st = np.zeros(3, np.int64)
    lx, ly, lm = _f64(lenses.x), _f64(lenses.y), _f64(lenses.m)
    cs = np.ascontiguousarray(cell_start, np.int64)
    pm = np.ascontiguousarray(perm, np.int64)
    lib.orc_shoot_interp_rays(C.byref(s), lenses.n, _ptr(lx), _ptr(ly), _ptr(lm), _ptr(cs),
                              _ptr(pm), first, n, _ptr(ray_ids), _ptr(ax), _ptr(ay), _ptr(pix),
                              _ptr(counts), _ptr(st), threads)
    return dict(alpha1=ax, alpha2=ay, pix=pix, counts=counts, landed=int(st[0]),
                off=int(st[1]), singular=int(st[2]))


def sheet_taylor(g: Geometry, z0: complex):
    """g_0 = F(z0) and g_k = G^(k)(z0)/k!, k = 1..4, of the sheet function
    F = (I1 - i I2)/pi.  Pinned by the 5th-order convergence of
    F(z0+h) - [g0 + conj(h) + sum g_k h^k] and finite differences of F."""
    lib = load()
    s = setup_of(g)
    out = np.empty(10)
    lib.orc_sheet_taylor_xy(C.byref(s), float(z0.real), float(z0.imag), _ptr(out))
    return out[0::2] + 1j * out[1::2]


def far_point(g: Geometry, lenses, cell_start, perm, cx, cy, x, y, threads=0):
    """Analytic far field A and its derivative A' of cell (cx[k], cy[k]) at the
    points (x[k], y[k]) (orc_far_point).  Returns complex arrays (A, dA).

    Pinned by: the direct definition (O-1) at the same points, since
    conj(alpha - macro - near) = A - kappa_* conj(z) outside the corner cells,
    and by central differences of A for A'."""
    lib = load()
    s = setup_of(g)
    cx = np.ascontiguousarray(cx, dtype=np.int64)
    cy = np.ascontiguousarray(cy, dtype=np.int64)
    x, y = _f64(x), _f64(y)
    n = cx.size
    out = np.zeros(4 * n)
    lx, ly, lm = _f64(lenses.x), _f64(lenses.y), _f64(lenses.m)
    cs = np.ascontiguousarray(cell_start, dtype=np.int64)
    pm = np.ascontiguousarray(perm, dtype=np.int64)
    lib.orc_far_point(C.byref(s), lenses.n, _ptr(lx), _ptr(ly), _ptr(lm),
                      _ptr(cs), _ptr(pm), n, _ptr(cx), _ptr(cy), _ptr(x), _ptr(y), _ptr(out),
                      threads)
    o = out.reshape(n, 4)
    return o[:, 0] + 1j * o[:, 1], o[:, 2] + 1j * o[:, 3]
