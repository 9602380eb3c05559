"""Every entry point of the C oracle on a small workload, with digests of the
results, to compare two builds of it (the sanitizer build against the
regular one)."""
import hashlib

import numpy as np

import oracle as orc
import synth


def _digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        if a is None:
            h.update(b"none")
        else:
            a = np.ascontiguousarray(a)
            h.update(str(a.dtype).encode())
            h.update(a.tobytes())
    return h.hexdigest()


def run():
    out = {}
    for tag, mass, sheet in (("unit", "unit", True), ("salpeter", "salpeter", True),
                             ("no sheet", "unit", False)):
        g = orc.geometry(0.45, 0.05, 0.45, 2.0, 16, n_rays=4_000, sheet=sheet,
                         level2_ray_multiple=0.5)
        L = synth.uniform_lenses(g.n_stars_expected, g.rect, 3, mass=mass)
        g = g.with_lens_count(L.n)
        d = orc.shoot_direct(g, L, threads=2)
        out[f"direct {tag}"] = [_digest(d["alpha1"], d["alpha2"], d["pix"], d["counts"]),
                                d["landed"], d["off"], d["singular"]]
        ids = np.arange(0, g.nx * g.ny, 97, dtype=np.int64)
        d = orc.shoot_direct(g, L, ray_ids=ids, threads=2)
        out[f"direct ids {tag}"] = _digest(d["alpha1"], d["alpha2"], d["pix"])
        cs, perm = orc.level1(g, L)
        out[f"level1 {tag}"] = _digest(cs, perm)
        coef = orc.level2_grid(g, L, cs, perm, threads=2)
        out[f"level2 grid {tag}"] = _digest(coef)
        gx = np.arange(0, g.n1x * g.q, 7, dtype=np.int64)
        gy = (gx * 3) % (g.n1y * g.q)
        out[f"level2 points {tag}"] = _digest(orc.level2(g, L, cs, perm, gx, gy, threads=2))
        d = orc.shoot_interp(g, L, cs, perm, coef, threads=2)
        out[f"interp {tag}"] = [_digest(d["alpha1"], d["alpha2"], d["pix"], d["counts"]),
                                d["landed"], d["off"]]
        d = orc.shoot_interp_rays(g, L, cs, perm, ray_ids=ids, threads=2)
        out[f"interp rays {tag}"] = _digest(d["alpha1"], d["alpha2"], d["pix"])
        x = np.linspace(g.a1, g.a2, 101)
        y = np.linspace(g.b1, g.b2, 101)[::-1].copy()
        a1, a2, ns = orc.alpha_points(g, L, x, y)
        out[f"alpha points {tag}"] = [_digest(a1, a2), ns]
        cx = np.arange(101, dtype=np.int64) % g.n1x
        cy = (np.arange(101, dtype=np.int64) * 5) % g.n1y
        fx = g.a1 + (cx + 0.37) * (g.a2 - g.a1) / g.n1x          # points inside their cells
        fy = g.b1 + (cy + 0.61) * (g.b2 - g.b1) / g.n1y
        A, dA = orc.far_point(g, L, cs, perm, cx, cy, fx, fy, threads=2)
        out[f"far point {tag}"] = _digest(A, dA)
        if sheet:
            out[f"sheet taylor {tag}"] = _digest(orc.sheet_taylor(g, complex(0.3, -0.2)))
    I1, I2 = orc.sheet_I((-2.0, 3.0, -1.0, 1.5), np.linspace(-5, 5, 77), np.linspace(-3, 3, 77))
    out["sheet I"] = _digest(I1, I2)
    return out
