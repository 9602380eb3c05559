"""Accuracy against the number of rays (Sec. 3.2, reduced in size): maps of a
regular ray grid converge to a high-ray reference with a logarithmic slope
between the Poisson -1/2 and the -3/4 of uniform grids (the paper reports
about -2/3), and every finer map is closer to the reference.  The reference
is the direct sum (FP32 with compensation, 1.6e9 rays), itself checked on a
seeded ray sample against the FP64 oracle's direct definition."""
import numpy as np
import pytest

import oracle as orc
import synth
from gpu_common import THREADS, rel_err

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
    kw = dict(kappa_star=0.652, kappa_c=0.0, gamma=0.0, source_side=S, npix=npix)
    p0 = irs.make_params(**kw, n_rays=1, method="interp", precision="fp64")
    g0 = irs.geometry(p0, 0)
    L = synth.uniform_lenses(g0["n_stars_expected"], (g0["a1"], g0["a2"], g0["b1"], g0["b2"]), 808)

    def shoot(n_rays, method="interp", precision="fp64"):
        p = irs.make_params(**kw, n_rays=n_rays, method=method, precision=precision)
        pl = irs.Plan(p, L.x, L.y, L.m)
        c, st = pl.shoot_map()
        return c, pl

    # the reference: the direct sum over every lens for 1.6e9 rays
    ref, pref = shoot(40_000 ** 2, "direct", "fp32")
    s_ref = pref.geometry["s_img"]
    rng = np.random.default_rng(21)
    ids = np.sort(rng.choice(pref.n_rays, 2000, replace=False))
    got = [pref.deflect_grid(int(r), 1) for r in ids]
    a1 = np.array([g[0][0] for g in got])
    a2 = np.array([g[1][0] for g in got])
    px = np.array([g[2][0] for g in got])
    pref.close()
    og = orc.geometry(**kw, n_rays=40_000 ** 2).with_lens_count(L.n)
    o1 = orc.shoot_direct(og, L, ray_ids=ids, threads=THREADS, want_counts=False)
    e = rel_err(a1, a2, o1["alpha1"], o1["alpha2"])
    say(f"reference: {L.n} lenses, 1.6e9 rays, direct FP32; sample of 2000 rays vs O-1: "
        f"max e_r {e.max():.2e}, pixel mismatches {int(np.sum(px != o1['pix']))}")
    assert np.mean(e <= 1e-5) >= 0.9999
    assert np.sum(px != o1["pix"]) <= 1

    total = []
    slopes = []
    for k in (1, 2, 3, 4):
        m, pl = shoot((2560 * k) ** 2)
        s = pl.geometry["s_img"]
        pl.close()
        x, rms, n, tot = rms_by_rays(m, ref, s, s_ref)
        sel = (x > 10) & (n >= 50)
        slope = float(np.polyfit(np.log10(x[sel]), np.log10(rms[sel]), 1)[0])
        say(f"{(2560 * k) ** 2:.3e} rays: overall RMS {tot:.3e}, slope {slope:.3f}")
        total.append(tot)
        slopes.append(slope)
    assert all(a > b for a, b in zip(total, total[1:]))
    assert all(-0.9 < s < -0.45 for s in slopes), slopes
