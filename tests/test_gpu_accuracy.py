"""Accuracy against the number of rays (Sec. 3.2, reduced in size): maps of a
regular ray grid converge to a high-ray reference with a logarithmic slope
between the Poisson -1/2 and the -3/4 of uniform grids (the paper reports
about -2/3), and every finer map is closer to the reference."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def rms_by_rays(test, ref, s_test, s_ref, nbins=100):
    t = test.astype(np.float64).ravel()
    r = ref.astype(np.float64).ravel()
    ok = (t > 0) & (r > 0)
    t, r = t[ok], r[ok]
    err = (t * s_test) / (r * s_ref) - 1.0
    edges = np.logspace(np.log10(t.min()), np.log10(t.max() + 1), nbins + 1)
    idx = np.clip(np.digitize(t, edges) - 1, 0, nbins - 1)
    n = np.bincount(idx, minlength=nbins)
    ss = np.bincount(idx, weights=err * err, minlength=nbins)
    sn = np.bincount(idx, weights=t, minlength=nbins)
    keep = n >= 20
    return sn[keep] / n[keep], np.sqrt(ss[keep] / n[keep]), n[keep], float(np.sqrt(np.mean(err * err)))


def test_error_falls_with_rays_at_a_uniform_grid_slope():
    import paper_2204_10871_amd as irs
    irs.load()
    S, npix = 40.0, 256
    p0 = irs.make_params(0.652, 0.0, 0.0, S, npix, n_rays=1, method="interp", precision="fp64")
    g0 = irs.geometry(p0, 0)
    L = synth.uniform_lenses(g0["n_stars_expected"], (g0["a1"], g0["a2"], g0["b1"], g0["b2"]), 808)

    def shoot(n_rays):
        p = irs.make_params(0.652, 0.0, 0.0, S, npix, n_rays=n_rays, method="interp",
                            precision="fp64")
        with irs.Plan(p, L.x, L.y, L.m) as pl:
            c, st = pl.shoot_map()
            return c, pl.geometry["s_img"]

    ref, s_ref = shoot(40_000 ** 2)
    total = []
    slopes = []
    for k in (1, 2, 3, 4):
        m, s = shoot((2560 * k) ** 2)
        x, rms, n, tot = rms_by_rays(m, ref, s, s_ref)
        sel = (x > 10) & (n >= 50)
        slope = float(np.polyfit(np.log10(x[sel]), np.log10(rms[sel]), 1)[0])
        say(f"{(2560 * k) ** 2:.3e} rays: overall RMS {tot:.3e}, slope {slope:.3f}")
        total.append(tot)
        slopes.append(slope)
    assert all(a > b for a, b in zip(total, total[1:]))
    assert all(-0.9 < s < -0.45 for s in slopes), slopes
