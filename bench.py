#!/usr/bin/env python3
"""Benchmark of the inverse-ray-shooting hot path on one MI355X.

Workload: the large-regime map -- kappa_* = gamma = 0.6, kappa_c = 0,
N_* = 1e6 lenses with Salpeter masses on [0.1, 1] M_sun, a 10000^2 pixel
source map and 1000 rays per pixel (1e11 rays over a 5117 x 1023 theta_E
rectangle).  Inputs are seeded and synthetic and resident in HBM before the
timed region.

One step = one whole map through the interpolated path (Sec. 2.4): every
distant-field expansion and level-2 coefficient band recomputed (FP64), then
every ray (near lenses exactly, distant lenses and the sheet by the Taylor
series, macro term, binning into the device-resident count map).

Printed: one JSON line (stdout) with the whole-job throughput in rays/s; the
roofline of the dominant kernel, k_level3 (the level-3 rays, FP64 VALU), from
HIP-event timings of its launches on the plan's stream; the parity sample
(1e5 rays drawn over the whole map plus 1e4 rays near lenses, against the
FP64 oracle's direct definition: per-ray error, index agreement, the map
rel-L1 bound); the oracle's CPU baseline (median of three timed runs on that
sample); and the FP32 direct sum at N_* = 1e6 with its own error against the
oracle.  Optional sections: accuracy against rays (Sec. 3.2), the learned
interpolant, the 64-map batch, the protective border, the circular plane.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/sec and ray-lens interactions/sec at N_*=1e6; map rel-L1 vs FP64 oracle"
FP64_PEAK = 78.6     # TFLOP/s, MI355X vector FP64
FP32_PEAK = 157.3    # TFLOP/s, MI355X vector FP32 (packed)
DIRECT_FLOPS_PER_PAIR = 11
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "level3_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2204_10871_amd", "csrc", "k_interp.hip")


def _traffic(launches):
    """HBM bytes per launch of k_level3 from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), or None when
    there is none or the kernel source has changed since it was taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bench_learned(irs, synth, torch, stream, args, result):
    """The learned interpolant on its workload (kappa_* = gamma = 0.5,
    kappa_c = 0.05, N_* = 1e6 unit lenses, 8192^2 px, 100 rays/px): training,
    validation, three level-1 row bands timed against the grid interpolation
    on the same bands, and a ray sample checked against the oracle's direct sum."""
    import numpy as np
    import oracle as orc
    w = synth.configs.CFG5
    pL = irs.params_from_workload(w, method="learned", precision="fp64")
    pI = irs.params_from_workload(w, method="interp", precision="fp64")
    g0 = irs.geometry(pL, 0)
    L = synth.uniform_lenses(g0["n_stars_expected"], (g0["a1"], g0["a2"], g0["b1"], g0["b2"]),
                             w.seed)
    out = {"workload": "kappa*=0.5 kappa_c=0.05 gamma=0.5, N*=1e6 unit, S=532.16, 8192^2 px, "
                       "N_av=100 (6.7e9 rays)", "n_star": L.n}
    npix = w.npix
    counts = torch.zeros(npix * npix, dtype=torch.int32, device="cuda:0")
    with irs.Plan(pL, L.x, L.y, L.m, stream=stream.cuda_stream) as pl, \
            irs.Plan(pI, L.x, L.y, L.m, stream=stream.cuda_stream) as pi:
        G = pl.geometry
        t0 = time.perf_counter()
        rep = pl.learn(synth.network.fourier_frequencies(7), irs.learn_params())
        out["learn_seconds"] = time.perf_counter() - t0
        out["report"] = rep
        log(f"learned: trained in {out['learn_seconds']:.1f} s, val mean |err| "
            f"{rep['val_mean_abs']:.2e} (grid alone {rep['base_mean_abs']:.2e}, tol "
            f"{rep['tol_mean']:.2e}), fallback {rep['fallback']}")
        c_mid = G["n1y"] // 2
        bands = [pl.level1_row_rays(c_mid)]
        res = {}
        for name, plan in (("learned", pl), ("interp", pi)):
            j0, j1 = pl.level1_row_rays(c_mid - 1)
            plan.shoot_rows(j0, j1 - j0, counts)                 # loads the kernels
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = plan.shoot_map_device(counts, time_phases=True)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t1
            res[name] = {"full_map_seconds": sec, "rays_per_s": st["rays_shot"] / sec,
                         "ms_level2": st["ms_level2"], "ms_level2_expansions": st["ms_level2_expand"],
                         "ms_rays": st["ms_rays"], "learned_used": st["learned"]}
            log(f"{name}: whole map {sec:.2f} s (level-2 {st['ms_level2']:.0f} ms, rays "
                f"{st['ms_rays']:.0f} ms), {st['rays_shot'] / sec:.3e} rays/s")
        out.update(res)
        # check: the direct definition on a ray sample of the first band
        og = orc.geometry(w.kappa_star, w.kappa_c, w.gamma, w.source_side, w.npix,
                          rays_per_pixel=w.rays_per_pixel, n_lens=L.n)
        j0, j1 = bands[0]
        rng = np.random.default_rng(11)
        nsamp = 4000
        ids = np.sort(rng.choice((j1 - j0) * G["nx"], nsamp, replace=False)) + j0 * G["nx"]
        threads = min(16, os.cpu_count() or 1)
        ref = orc.shoot_direct(og, L, ray_ids=ids, threads=threads, want_counts=False)
        for name, plan in (("learned", pl), ("interp", pi)):
            n = (j1 - j0) * G["nx"]
            a1 = torch.empty(n, dtype=torch.float64, device="cuda:0")
            a2 = torch.empty(n, dtype=torch.float64, device="cuda:0")
            px = torch.empty(n, dtype=torch.int64, device="cuda:0")
            plan.deflect_grid_device(j0 * G["nx"], n, a1, a2, px)
            sel = torch.as_tensor(ids - j0 * G["nx"], device="cuda:0")
            g1, g2, gp = a1[sel].cpu().numpy(), a2[sel].cpu().numpy(), px[sel].cpu().numpy()
            d = np.hypot(g1 - ref["alpha1"], g2 - ref["alpha2"])
            rel = d / np.hypot(ref["alpha1"], ref["alpha2"])
            mis = int(np.sum(gp != ref["pix"]))
            out[name]["direct_check"] = {"rays": int(nsamp), "max_abs_alpha_err": float(d.max()),
                                  "mean_abs_alpha_err": float(d.mean()),
                                  "max_rel_alpha_err": float(rel.max()),
                                  "pixel_mismatches": mis}
            log(f"{name} vs direct on {nsamp} rays: max |d alpha| {d.max():.2e}, "
                f"pixel mismatches {mis}")
        direct = result.get("direct_fp32", {}).get("interactions_per_s")
        if direct:
            t_direct = G["nx"] * G["ny"] * L.n / direct
            out["direct_fp32_full_map_seconds_estimated"] = t_direct
            for name in ("learned", "interp"):
                out[name]["speedup_over_direct"] = t_direct / out[name]["full_map_seconds"]
        out["coefficient_bytes_per_level1_row"] = {"learned": rep["corner_bytes_per_row"],
                                                   "interp": rep["coef_bytes_per_row"]}
    return out


def rms_by_rays(test, ref, s_test, s_ref, nbins=300):
    """Pixel-by-pixel relative error of the magnification (N S_I / S_S) of a
    map against a reference, RMS in logarithmic bins of the map's rays per
    pixel (Sec. 3.2).  Returns (bin centres, RMS, pixels per bin)."""
    import numpy as np
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
    return sn[keep] / n[keep], np.sqrt(ss[keep] / n[keep]), n[keep]


def bench_accuracy(irs, synth, torch, stream):
    """Accuracy against the number of rays (Sec. 3.2): kappa = kappa_* = 0.652,
    gamma = 0, 1024^2 px, equal masses, S = 50 Einstein radii of a solar mass
    with <M> = 0.1 solar masses (158.1 in units of the mean mass); maps of
    (10240 k)^2 rays, k = 1..7, against a 4e10-ray map of the same lenses; RMS
    relative magnification error in 300 logarithmic bins of rays per pixel and
    the slope of log RMS against log rays per pixel.  The reference map is the
    interpolated path at 4e10 rays (a direct sum over the ~52,000 lenses would
    take ~400 s); the test of this experiment uses a direct-sum reference at a
    smaller size."""
    import numpy as np
    S = 50.0 / math.sqrt(0.1)
    npix = 1024
    p0 = irs.make_params(0.652, 0.0, 0.0, S, npix, n_rays=1, method="interp", precision="fp64")
    g0 = irs.geometry(p0, 0)
    L = synth.uniform_lenses(g0["n_stars_expected"], (g0["a1"], g0["a2"], g0["b1"], g0["b2"]),
                             synth.configs.SEED_BASE + 8)
    counts = torch.zeros(npix * npix, dtype=torch.int32, device="cuda:0")

    def shoot(n_rays):
        p = irs.make_params(0.652, 0.0, 0.0, S, npix, n_rays=n_rays, method="interp",
                            precision="fp64")
        with irs.Plan(p, L.x, L.y, L.m, stream=stream.cuda_stream) as pl:
            st = pl.shoot_map_device(counts)
            g = pl.geometry
        torch.cuda.synchronize()
        return counts.cpu().numpy().reshape(npix, npix).copy(), g["s_img"], st

    t0 = time.perf_counter()
    ref, s_ref, st_ref = shoot(200_000 ** 2)
    out = {"workload": "kappa=kappa_*=0.652, gamma=0, S=158.1 (mean-mass units), 1024^2 px, "
                       "equal masses, interpolated path", "n_star": L.n,
           "reference": "the interpolated path itself at 4e10 rays (not a direct sum)",
           "reference_rays": st_ref["rays_shot"], "maps": []}
    slopes = []
    for k in range(1, 8):
        m, s_img, st = shoot((10240 * k) ** 2)
        x, rms, n = rms_by_rays(m, ref, s_img, s_ref)
        sel = (x > 10) & (n >= 100)
        slope = float(np.polyfit(np.log10(x[sel]), np.log10(rms[sel]), 1)[0]) if sel.sum() > 3 else None
        slopes.append(slope)
        out["maps"].append({"rays": st["rays_shot"], "mean_rays_per_pixel": float(m.mean()),
                            "slope": slope, "rms_at_median": float(np.median(rms))})
        log(f"accuracy: {st['rays_shot']:.3e} rays, slope {slope:.3f}, median RMS {np.median(rms):.3e}")
    good = [s for s in slopes if s is not None]
    out["slope_mean"] = float(np.mean(good)) if good else None
    out["seconds"] = time.perf_counter() - t0
    return out


def _ray_thetas(g, torch, r0, n):
    """theta of rays r0 .. r0+n-1 of a plan (row-major grid, rays at cell centres)."""
    r = torch.arange(r0, r0 + n, dtype=torch.int64, device="cuda:0")
    i, j = r % g["nx"], r // g["nx"]
    return (g["a1"] + (i.double() + 0.5) * g["ray_dx"], g["b1"] + (j.double() + 0.5) * g["ray_dy"])


def border_coverage(irs, synth, torch, stream, kappa_star, kappa_c, gamma, S, npix,
                    rays_per_pixel, seed, big=3.0, mass="unit", chunk=1 << 24):
    """The protective border's ray coverage (Sec. 2.3): with border P = 10
    sqrt(kappa_*) the shooting rectangle holds a fraction of the rays that
    reach the target map; the rest start beyond it.  A plan with border big*P
    and the same ray spacing and lens density stands in for the unbounded
    plane: coverage = (its map-landing rays that start inside the border-P
    rectangle) / (all its map-landing rays).  FP64 direct sum."""
    P = 10.0 * math.sqrt(kappa_star)
    g_in = irs.geometry(irs.make_params(kappa_star, kappa_c, gamma, S, npix,
                                        rays_per_pixel=rays_per_pixel), 0)
    dx3 = g_in["dx3"]
    g0 = irs.geometry(irs.make_params(kappa_star, kappa_c, gamma, S, npix, n_rays=1,
                                      border=big * P), 0)
    n_big = int(round((g0["a2"] - g0["a1"]) * (g0["b2"] - g0["b1"]) / (dx3 * dx3)))
    p = irs.make_params(kappa_star, kappa_c, gamma, S, npix, n_rays=n_big, border=big * P,
                        method="direct", precision="fp64")
    g = irs.geometry(p, 0)
    L = synth.uniform_lenses(g["n_stars_expected"], (g["a1"], g["a2"], g["b1"], g["b2"]), seed,
                             mass=mass)
    total = g["nx"] * g["ny"]
    px = torch.empty(min(chunk, total), dtype=torch.int64, device="cuda:0")
    landed = inner = 0
    t0 = time.perf_counter()
    with irs.Plan(p, L.x, L.y, L.m, stream=stream.cuda_stream) as pl:
        for r0 in range(0, total, chunk):
            n = min(chunk, total - r0)
            pl.deflect_grid_device(r0, n, None, None, px[:n])
            t1, t2 = _ray_thetas(g, torch, r0, n)
            hit = px[:n] >= 0
            ins = (t1 >= g_in["a1"]) & (t1 < g_in["a2"]) & (t2 >= g_in["b1"]) & (t2 < g_in["b2"])
            landed += int(hit.sum())
            inner += int((hit & ins).sum())
    torch.cuda.synchronize()
    return {"kappa_star": kappa_star, "kappa_c": kappa_c, "gamma": gamma, "source_side": S,
            "npix": npix, "border": P, "outer_border": big * P, "n_star_outer": L.n,
            "rays_outer": total, "landed": landed, "landed_from_inside": inner,
            "coverage": inner / landed if landed else None,
            "seconds": time.perf_counter() - t0}


def perturbation_u(irs, synth, torch, stream, n_star, realizations, spacing, seed0,
                   kappa_star=0.5, central=0.5):
    """|phi|/phi_0 of the stars' deflection perturbation (deflection of n_star
    unit masses plus the negative sheet, i.e. alpha minus the macro term
    kappa_* theta at kappa_c = gamma = 0), sampled on a grid of spacing
    `spacing` over the central `central` fraction (per side) of a square lens
    plane holding exactly n_star lenses at density kappa_*; `realizations`
    independent lens draws.  FP64 direct sum.  Returns a host array."""
    import numpy as np
    side = math.sqrt(math.pi * n_star / kappa_star)
    S = side * (1.0 - kappa_star)                     # border 0: the plane is S/(1 - kappa_*)
    n_rays = int(round((side / spacing) ** 2))
    p = irs.make_params(kappa_star, 0.0, 0.0, S, 64, n_rays=n_rays, border=0.0,
                        method="direct", precision="fp64")
    g = irs.geometry(p, 0)
    total = g["nx"] * g["ny"]
    a1 = torch.empty(total, dtype=torch.float64, device="cuda:0")
    a2 = torch.empty_like(a1)
    t1, t2 = _ray_thetas(g, torch, 0, total)
    half = 0.5 * central * side
    sel = (t1.abs() <= half) & (t2.abs() <= half)
    out = []
    for r in range(realizations):
        L = synth.uniform_lenses(n_star, (g["a1"], g["a2"], g["b1"], g["b2"]), seed0 + r)
        with irs.Plan(p, L.x, L.y, L.m, stream=stream.cuda_stream) as pl:
            pl.deflect_grid_device(0, total, a1, a2, None)
            u = torch.sqrt((a1 - kappa_star * t1) ** 2 + (a2 - kappa_star * t2) ** 2)[sel]
            out.append((u / math.sqrt(kappa_star)).cpu().numpy())
    return np.concatenate(out)


def bench_border(irs, synth, torch, stream):
    """Protective border and deflection-perturbation density (Sec. 2.3): the
    coverage of the 10 sqrt(kappa_*) border on three lens-plane shapes, and the
    measured density of |phi|/phi_0 against the closed forms with c = 3.05
    (Katz et al.) and c = 1.454 (the paper's modified form): Kolmogorov-Smirnov
    distance of the radial CDFs."""
    import numpy as np
    from oracle import border as ob
    t0 = time.perf_counter()
    out = {"coverage": [], "perturbation": []}
    for (ks, kc, gm, S, npix, rpp, seed) in ((0.3, 0.0, 0.3, 10.0, 256, 64.0, 901),
                                             (0.45, 0.05, 0.45, 25.0, 1024, 4.0, 902),
                                             (0.6, 0.0, 0.6, 50.0, 512, 16.0, 903)):
        c = border_coverage(irs, synth, torch, stream, ks, kc, gm, S, npix, rpp, seed)
        out["coverage"].append(c)
        log(f"border: kappa_*={ks} kappa_c={kc} gamma={gm} S={S}: coverage {c['coverage']:.5f} "
            f"({c['landed']:.3e} landed rays, {c['n_star_outer']} lenses)")
    ugrid = np.concatenate([np.linspace(0.05, 8.0, 160), np.geomspace(8.2, 40.0, 24)])
    # ~900 samples per draw (a 30 x 30 grid over the central half); the field's
    # long-range part is shared by a draw's samples, so the draws, not the
    # samples, set the statistical weight
    for n, reals in ((100, 400), (1000, 300), (10000, 200), (100000, 100), (1000000, 40)):
        spacing = math.sqrt(math.pi * n / 0.5) * 0.5 / 30.0
        u = np.sort(perturbation_u(irs, synth, torch, stream, n, reals, spacing, 1000 * n))
        Femp = np.searchsorted(u, ugrid, side="right") / u.size
        rec = {"n_star": n, "realizations": reals, "samples": int(u.size), "spacing": spacing,
               "median": float(np.median(u)), "p98": float(np.quantile(u, 0.98))}
        for name, cc in (("katz", ob.KATZ_C), ("modified", ob.MODIFIED_C)):
            F = ob.radial_cdf(ugrid, n, cc)
            rec[f"ks_{name}"] = float(np.max(np.abs(Femp - F)))
            rec[f"median_{name}"] = float(ugrid[np.searchsorted(F, 0.5)])
        out["perturbation"].append(rec)
        log(f"border: N={n}: {u.size} samples, median |phi|/phi0 {rec['median']:.3f} "
            f"(Katz {rec['median_katz']:.3f}, modified {rec['median_modified']:.3f}), "
            f"KS distance Katz {rec['ks_katz']:.4f}, modified {rec['ks_modified']:.4f}")
    out["seconds"] = time.perf_counter() - t0
    return out


def bench_circle(irs, synth, torch, stream):
    """Circular against rectangular lens plane (Sec. 2.2): lenses needed for
    the paper's workloads (the circle circumscribes the image rectangle), and
    whole FP64 direct-sum maps of the kappa_* = gamma = 0.45, kappa_c = 0.05
    shape (aspect 19) with each plane."""
    out = {"lens_counts": []}
    for w in (synth.configs.CFG1, synth.configs.CFG2, synth.configs.CFG3, synth.configs.CFG5):
        kw = dict(kappa_star=w.kappa_star, kappa_c=w.kappa_c, gamma=w.gamma,
                  source_side=w.source_side, npix=w.npix, rays_per_pixel=w.rays_per_pixel,
                  n_rays=w.n_rays)
        gr = irs.geometry(irs.make_params(**kw), 0)
        gc = irs.geometry(irs.make_params(circle=True, **kw), 0)
        out["lens_counts"].append({"workload": w.name, "aspect": gr["ix"] / gr["iy"],
                                   "rectangle": gr["n_stars_expected"],
                                   "circle": gc["n_stars_expected"],
                                   "ratio": gc["n_stars_expected"] / gr["n_stars_expected"]})
        log(f"circle: {w.name}: {gr['n_stars_expected']} lenses (rectangle) against "
            f"{gc['n_stars_expected']} (circle), x{gc['n_stars_expected'] / gr['n_stars_expected']:.2f}")
    npix = 1024
    counts = torch.zeros(npix * npix, dtype=torch.int32, device="cuda:0")
    timing = {}
    for circle in (False, True):
        p = irs.make_params(0.45, 0.05, 0.45, 25.0, npix, rays_per_pixel=4.0, circle=circle,
                            method="direct", precision="fp64")
        g = irs.geometry(p, 0)
        if circle:
            L = synth.disc_lenses(g["n_stars_expected"], g["lens_radius"], 905)
        else:
            L = synth.uniform_lenses(g["n_stars_expected"], (g["a1"], g["a2"], g["b1"], g["b2"]), 905)
        with irs.Plan(p, L.x, L.y, L.m, stream=stream.cuda_stream) as pl:
            pl.shoot_map_device(counts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = pl.shoot_map_device(counts)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
        key = "circle" if circle else "rectangle"
        timing[key] = {"lenses": L.n, "rays": st["rays_shot"], "landed": st["rays_landed"],
                       "seconds": sec, "pairs_per_s": st["rays_shot"] * L.n / sec}
        log(f"circle: {key} plane, {L.n} lenses, {st['rays_shot']:.3e} rays: {sec * 1e3:.1f} ms "
            f"({st['rays_shot'] * L.n / sec:.3e} pairs/s)")
    timing["time_ratio"] = timing["circle"]["seconds"] / timing["rectangle"]["seconds"]
    out["fp64_direct_aspect19"] = timing
    return out


def _batch_plans(irs, synth, torch, stream, method, precision, rays_per_pixel=None):
    draws = synth.configs.batch_draws()
    plans, counts = [], []
    for d in draws:
        S = irs.source_side_for_n_star(d.kappa_star, d.kappa_c, d.gamma, d.n_star_target)
        rpp = d.rays_per_pixel if rays_per_pixel is None else rays_per_pixel
        p = irs.make_params(d.kappa_star, d.kappa_c, d.gamma, S, d.npix, rays_per_pixel=rpp,
                            method=method, precision=precision)
        g = irs.geometry(p, 0)
        L = synth.uniform_lenses(g["n_stars_expected"], (g["a1"], g["a2"], g["b1"], g["b2"]),
                                 d.seed)
        plans.append(irs.Plan(p, L.x, L.y, L.m, stream=stream.cuda_stream))
        counts.append(torch.empty(d.npix * d.npix, dtype=torch.int32, device="cuda:0"))
    return plans, counts


def _batch_vs_sequential(irs, torch, plans, counts, repeats=3):
    """(tuned settings, graph seconds, one-by-one seconds, identical maps);
    each time the median of `repeats` runs."""
    def timed(f):
        torch.cuda.synchronize()
        t = time.perf_counter()
        f()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    with irs.Batch(plans) as b:
        info = b.tune()
        b.run(counts)                                      # capture + first replay
        tb = statistics.median(timed(lambda: b.run(counts)) for _ in range(repeats))
    batched = [c.clone() for c in counts]

    def one_by_one():
        for p, c in zip(plans, counts):
            p.shoot_map_device(c)        # computes every expansion, as the graph does

    ts = statistics.median(timed(one_by_one) for _ in range(repeats))
    same = all(torch.equal(a, c) for a, c in zip(batched, counts))
    return info, tb, ts, same


def bench_batch(irs, synth, torch, stream):
    """The 64-map batch (kappa_*, gamma ~ U[0.1, 0.8], kappa_c in {0, 0.2},
    N_* = 10^U[3, 5], 1024^2..4096^2 px): one tuned graph launch against the
    same maps launched one after another.  Interpolated at 100 rays/px (every
    map's level 2, then one level-3 launch over every map's tiles); and the FP32 direct sum
    with the tuner's tile shape, at 1 ray/px (the stated 100 rays/px would
    take ~190 s of direct sums)."""
    out = {}
    t0 = time.perf_counter()
    plans, counts = _batch_plans(irs, synth, torch, stream, "interp", "fp64")
    rays = sum(p.n_rays for p in plans)
    log(f"batch: {len(plans)} maps, {rays:.3e} rays, set up in {time.perf_counter() - t0:.1f} s")
    info, tb, ts, same = _batch_vs_sequential(irs, torch, plans, counts)
    for p in plans:
        p.close()
    log(f"batch interp: graph {tb:.3f} s, one by one {ts:.3f} s, identical {same}, {info}")
    out.update({"maps": len(plans), "rays": rays, "method": "interp", "precision": "fp64",
                "batched_rays_per_s": rays / tb, "sequential_rays_per_s": rays / ts,
                "seconds_batched": tb, "seconds_sequential": ts,
                "speedup": ts / tb, "identical_to_sequential": same, "tuned": info})
    plans, counts = _batch_plans(irs, synth, torch, stream, "direct", "fp32", rays_per_pixel=1.0)
    rays_d = sum(p.n_rays for p in plans)
    pairs = sum(p.n_rays * p.geometry["n_lens"] for p in plans)
    info, tb, ts, same = _batch_vs_sequential(irs, torch, plans, counts)
    for p in plans:
        p.close()
    log(f"batch direct fp32 (1 ray/px): graph {tb:.3f} s, one by one {ts:.3f} s, "
        f"identical {same}, {pairs / tb:.3e} pairs/s, {info}")
    out["direct_fp32"] = {"rays_per_pixel": 1.0, "rays": rays_d, "pairs": pairs,
                          "seconds_batched": tb, "seconds_sequential": ts,
                          "batched_pairs_per_s": pairs / tb, "speedup": ts / tb,
                          "identical_to_sequential": same, "tuned": info,
                          "note": "N_av reduced from 100 to 1 so that the direct sums fit the run"}
    return out


def host_threads():
    """OpenMP threads for the oracle: the host share of one GPU."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_info():
    """CPU model, logical CPUs and physical cores of the host (/proc/cpuinfo)."""
    model, cores = None, set()
    phys = core = None
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and model is None:
                model = v
            elif k == "physical id":
                phys = v
            elif k == "core id":
                core = v
            elif not k and phys is not None and core is not None:
                cores.add((phys, core))
                phys = core = None
    except OSError:
        pass
    if phys is not None and core is not None:
        cores.add((phys, core))
    return {"model": model, "logical": os.cpu_count(), "physical": len(cores) or None}


def wilson_upper(k, n, z=1.96):
    """95% upper bound (Wilson) on a binomial fraction with k of n observed."""
    ph = k / n
    return (ph + z * z / (2 * n) + z * math.sqrt(ph * (1 - ph) / n + z * z / (4 * n * n))) / \
        (1 + z * z / n)


def sample_errors(a1, a2, px, r1, r2, rpx):
    """Per-ray relative deflection error e_r = |d alpha|/max(|alpha_ref|, 1)
    and index agreement of a ray sample against the oracle."""
    import numpy as np
    d = np.hypot(a1 - r1, a2 - r2)
    e = d / np.maximum(np.hypot(r1, r2), 1.0)
    mism = int(np.sum(px != rpx))
    return {"max_e_r": float(e.max()), "p9999_e_r": float(np.quantile(e, 0.9999)),
            "max_abs_alpha_err": float(d.max()), "index_mismatches": mism,
            "agreement": 1.0 - mism / px.size}


def near_lens_rays(G, L, n, radius, rng):
    """n ray ids whose ray lies within `radius` of a lens: a random lens, a
    random point within radius - (half a ray-cell diagonal) of it, and the
    ray whose cell holds that point."""
    import numpy as np
    if n <= 0:
        return np.zeros(0, np.int64)
    half_diag = 0.5 * math.hypot(G["ray_dx"], G["ray_dy"])
    k = rng.integers(0, L.n, n)
    rad = (radius - half_diag) * np.sqrt(rng.random(n))
    ang = 2 * math.pi * rng.random(n)
    x = L.x[k] + rad * np.cos(ang)
    y = L.y[k] + rad * np.sin(ang)
    i = np.clip(np.floor((x - G["a1"]) / G["ray_dx"]).astype(np.int64), 0, G["nx"] - 1)
    j = np.clip(np.floor((y - G["b1"]) / G["ray_dy"]).astype(np.int64), 0, G["ny"] - 1)
    return np.unique(j * G["nx"] + i)


def gpu_rays(plan, ids):
    """alpha and pixel of listed rays (sorted ray order), one irs_deflect_grid
    call per ray."""
    import numpy as np
    a1 = np.empty(ids.size)
    a2 = np.empty(ids.size)
    px = np.empty(ids.size, np.int64)
    for k, r in enumerate(ids):
        x1, x2, p = plan.deflect_grid(int(r), 1)
        a1[k], a2[k], px[k] = x1[0], x2[0], p[0]
    return a1, a2, px


def direct_check(dplan, G, w, L, n_star, n, rays, landed, torch):
    """The FP32 direct sum against the oracle's direct definition: n rays
    drawn from 8 whole ray rows spread over the map (seeded), each row
    shot by one irs_deflect_grid call."""
    import numpy as np
    import oracle as orc
    rng = np.random.default_rng(8)
    nx = G["nx"]
    rows = np.sort(rng.choice(G["ny"], 8, replace=False))
    per = max(1, n // rows.size)
    a1 = torch.empty(nx, dtype=torch.float64, device="cuda:0")
    a2 = torch.empty_like(a1)
    px = torch.empty(nx, dtype=torch.int64, device="cuda:0")
    ids, g1, g2, gp = [], [], [], []
    for j in rows:
        dplan.deflect_grid_device(int(j) * nx, nx, a1, a2, px)
        cols = np.sort(rng.choice(nx, per, replace=False))
        sel = torch.as_tensor(cols, device="cuda:0")
        ids.append(int(j) * nx + cols)
        g1.append(a1[sel].cpu().numpy())
        g2.append(a2[sel].cpu().numpy())
        gp.append(px[sel].cpu().numpy())
    ids = np.concatenate(ids)
    og = orc.geometry(w.kappa_star, w.kappa_c, w.gamma, w.source_side, w.npix,
                      rays_per_pixel=w.rays_per_pixel, n_lens=n_star)
    ref = orc.shoot_direct(og, L, ray_ids=ids, threads=host_threads(), want_counts=False)
    out = sample_errors(np.concatenate(g1), np.concatenate(g2), np.concatenate(gp),
                        ref["alpha1"], ref["alpha2"], ref["pix"])
    up = wilson_upper(out["index_mismatches"], ids.size)
    out.update(rays=int(ids.size), ray_rows=[int(j) for j in rows], f_mis_95=up,
               map_rel_l1_bound=2 * up * rays / max(1, landed))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=100_000,
                    help="uniform rays of the parity sample / oracle baseline (each sums "
                         "all 1e6 lenses)")
    ap.add_argument("--near-sample", type=int, default=10_000,
                    help="extra parity rays within 0.05 theta_E of a lens")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--band-rows", type=int, default=0,
                    help="0: a step is the whole map; R > 0: a step is a band of R level-1 rows "
                         "(for counter runs)")
    ap.add_argument("--direct-rows", type=int, default=64)
    ap.add_argument("--direct-sample", type=int, default=100_000,
                    help="rays of the parity sample checked on the FP32 direct sum")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-map batch measurement")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the accuracy-versus-rays experiment (Sec. 3.2)")
    ap.add_argument("--no-circle", action="store_true",
                    help="skip the circular-against-rectangular lens plane section")
    ap.add_argument("--no-border", action="store_true",
                    help="skip the protective-border coverage and perturbation-density section")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-interpolant measurement (N_* = 1e6, 8192^2 px)")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="run a plain 512 MiB device copy first (scale for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2204_10871_amd as irs
    import synth

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    w = synth.configs.CFG3
    p = irs.params_from_workload(w, method="interp", precision="fp64")
    g0 = irs.geometry(p, 0)
    n_star = g0["n_stars_expected"]
    rect = (g0["a1"], g0["a2"], g0["b1"], g0["b2"])
    L = synth.uniform_lenses(n_star, rect, w.seed, mass=w.mass, m_min=w.m_min, m_max=w.m_max)
    plan = irs.Plan(p, L.x, L.y, L.m, stream=stream.cuda_stream)
    G = plan.geometry
    log(f"plan: {G['nx']}x{G['ny']} rays, N*={n_star}, level-1 {G['n1x']}x{G['n1y']}, q={G['q']}")
    counts = torch.zeros(w.npix * w.npix, dtype=torch.int32, device="cuda:0")

    if args.pmc_calibrate:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 512 MiB read + 512 MiB written")

    # a step: the whole map (every expansion recomputed: irs_shoot_map keeps
    # nothing from earlier calls), or a band of --band-rows level-1 rows
    c_mid = G["n1y"] // 2

    def step(k, timed):
        if args.band_rows > 0:
            c = c_mid + k * args.band_rows
            j0 = plan.level1_row_rays(c)[0]
            j1 = plan.level1_row_rays(min(G["n1y"] - 1, c + args.band_rows - 1))[1]
            counts.zero_()
            return plan.shoot_rows(j0, j1 - j0, counts, time_phases=timed)
        return plan.shoot_map_device(counts, time_phases=timed)

    for k in range(args.warmup):
        st = step(k, False)
        log(f"warmup {k}: {st['rays_shot']:.3e} rays, {st['ms_total']:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.warmup, args.warmup + args.steps):
        st = step(k, True)
        stats.append(st)
        log(f"step {k - args.warmup}: rays {st['rays_shot']:.3e} in {st['ms_total']:.1f} ms: "
            f"level-2 {st['ms_level2']:.1f} ms (expansions {st['ms_level2_expand']:.1f}), "
            f"level-3 {st['ms_rays']:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    rays = sum(s["rays_shot"] for s in stats)
    landed = sum(s["rays_landed"] for s in stats)
    value = rays / elapsed
    l2_pairs = sum(s["level2_pairs"] for s in stats)
    ex_flops = sum(s["level2_expand_flops"] for s in stats)
    ex_ms = sum(s["ms_level2_expand"] for s in stats)
    l2_ms = sum(s["ms_level2"] for s in stats)
    l3_ms = sum(s["ms_rays"] for s in stats)
    l3_flops = sum(s["ray_flops"] for s in stats)
    l3_launches = sum(s["n_ray_launches"] for s in stats)
    achieved = l3_flops / (l3_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK, 4),
                "traffic": _traffic(l3_launches),
                "kernel": "k_level3 (FP64 rays: Horner of the level-2 series, nearby lenses, "
                          "pixel, LDS-histogram binning)",
                "launches": l3_launches, "ms_per_launch": round(l3_ms / max(1, l3_launches), 3),
                "flops_per_launch": l3_flops / max(1, l3_launches)}
    phases = {"level2_ms_per_step": l2_ms / args.steps,
              "level2_expansions_ms_per_step": ex_ms / args.steps,
              "level2_expansions_tflops": ex_flops / max(ex_ms * 1e-3, 1e-12) / 1e12,
              "level3_ms_per_step": l3_ms / args.steps,
              "level2_all_kernels_tflops": sum(s["level2_flops"] for s in stats) / (l2_ms * 1e-3) / 1e12}
    step_name = ("the whole map (all level-1 row bands, every expansion)" if args.band_rows <= 0
                 else f"a band of {args.band_rows} level-1 rows")

    result = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "kappa*=0.6 kappa_c=0 gamma=0.6, N*=1e6 Salpeter [0.1,1] Msun, "
                               "10000^2 px, N_av=1000 (1e11 rays), interpolated "
                               "(level-2 FP64, dx2=dx1/20); step = " + step_name,
                   "n_star": n_star, "rays_per_step": rays / args.steps,
                   "method": "interp", "precision": "fp64"},
        "interactions_per_s": {"direct_equivalent": value * n_star,
                               "level2_point_lens_pairs_per_s": l2_pairs / elapsed},
        "full_map_seconds": G["nx"] * G["ny"] / value,
        "landed_fraction": landed / rays,
        "roofline": roofline,
        "phases": phases,
    }

    # ---- parity sample and the oracle's CPU baseline (rays it sums one by one)
    if not args.no_cpu_baseline:
        import oracle as orc
        threads = host_threads()
        og = orc.geometry(w.kappa_star, w.kappa_c, w.gamma, w.source_side, w.npix,
                          rays_per_pixel=w.rays_per_pixel, n_lens=n_star)
        assert og.nx == G["nx"] and og.ny == G["ny"]
        rng = np.random.default_rng(7)
        ids_u = np.sort(rng.choice(G["nx"] * G["ny"], args.cpu_sample, replace=False))
        ids_n = near_lens_rays(G, L, args.near_sample, 0.05, rng)
        tg = time.perf_counter()
        ga1, ga2, gpx = gpu_rays(plan, np.concatenate([ids_u, ids_n]))
        tg = time.perf_counter() - tg
        log(f"parity sample: {ids_u.size} uniform + {ids_n.size} near-lens rays from the GPU "
            f"in {tg:.1f} s; oracle on {threads} threads")
        # the uniform sample in three parts, each timed: the CPU baseline is the
        # median rate of the three runs
        parts, rates, tcpu = [], [], 0.0
        order = rng.permutation(ids_u.size)
        for chunk in np.array_split(order, 3):
            sel = np.sort(chunk)
            tc = time.perf_counter()
            parts.append((sel, orc.shoot_direct(og, L, ray_ids=ids_u[sel], threads=threads,
                                                want_counts=False)))
            dt = time.perf_counter() - tc
            tcpu += dt
            rates.append(sel.size / dt)
        ref_a1 = np.empty(ids_u.size)
        ref_a2 = np.empty(ids_u.size)
        ref_px = np.empty(ids_u.size, np.int64)
        for sel, r in parts:
            ref_a1[sel], ref_a2[sel], ref_px[sel] = r["alpha1"], r["alpha2"], r["pix"]
        refn = orc.shoot_direct(og, L, ray_ids=ids_n, threads=threads, want_counts=False)
        nu = ids_u.size
        uni = sample_errors(ga1[:nu], ga2[:nu], gpx[:nu], ref_a1, ref_a2, ref_px)
        near = sample_errors(ga1[nu:], ga2[nu:], gpx[nu:], refn["alpha1"], refn["alpha2"],
                             refn["pix"])
        up = wilson_upper(uni["index_mismatches"], nu)
        info = cpu_info()
        result["cpu_baseline"] = {
            "value": float(np.median(rates)), "unit": "rays/s", "cores": threads,
            "kind": "oracle",
            "sample": f"direct FP64 definition over all {n_star} lenses for {nu} rays drawn "
                      f"uniformly (seed 7) over all {G['nx'] * G['ny']} rays of this workload, "
                      f"timed as three runs of {nu // 3} rays; value = median rate; "
                      f"{tcpu:.1f} s in total",
            "runs_rays_per_s": rates, "cpu_model": info["model"],
            "box_logical_cpus": info["logical"], "box_physical_cores": info["physical"],
            "threads_note": "OpenMP threads = the host share of one GPU (OMP_NUM_THREADS, "
                            "else the CPUs this process may run on, at most 16)"}
        result["parity_sample"] = {
            "uniform": dict(uni, rays=nu, f_mis_95=up,
                            map_rel_l1_bound=2 * up * rays / max(1, landed)),
            "near_lens": dict(near, rays=int(ids_n.size), within_theta_E=0.05),
            "seconds_gpu": tg}
        log(f"parity: uniform {nu} rays: {uni['index_mismatches']} index mismatches "
            f"(95% bound {up:.2e}), max e_r {uni['max_e_r']:.2e}; near-lens {ids_n.size} rays: "
            f"{near['index_mismatches']} mismatches, max e_r {near['max_e_r']:.2e}")

    # ---- reference: the FP32 direct sum at N_* = 1e6 on a few tile rows, and
    # its per-ray error against the oracle on part of the parity sample
    if not args.no_direct:
        pd = irs.params_from_workload(w, method="direct", precision="fp32")
        with irs.Plan(pd, L.x, L.y, L.m, stream=stream.cuda_stream) as dplan:
            # whole tile rows (64 is a multiple of every tile height)
            r0 = (G["ny"] // 2) // 64 * 64
            rows = max(64, (args.direct_rows + 63) // 64 * 64)
            dplan.deflect_grid(r0 * G["nx"], 64)          # warm-up: one tile
            torch.cuda.synchronize()
            td = time.perf_counter()
            st = dplan.shoot_rows(r0, rows, counts, time_phases=True)
            torch.cuda.synchronize()
            td = time.perf_counter() - td
            check = None
            if not args.no_cpu_baseline and args.direct_sample > 0:
                check = direct_check(dplan, G, w, L, n_star, args.direct_sample, rays, landed,
                                     torch)
                log(f"direct fp32 vs oracle on {check['rays']} rays: max e_r "
                    f"{check['max_e_r']:.2e}, p99.99 {check['p9999_e_r']:.2e}, "
                    f"{check['index_mismatches']} index mismatches")
        pairs = st["direct_pairs"]
        tf = DIRECT_FLOPS_PER_PAIR * pairs / (st["ms_rays"] * 1e-3) / 1e12
        result["direct_fp32"] = {"rays_per_s": st["rays_shot"] / td,
                                 "interactions_per_s": pairs / td,
                                 "kernel_tflops_alg": tf, "frac_fp32_peak": tf / FP32_PEAK,
                                 "rays": st["rays_shot"], "seconds": td,
                                 "speedup_interp_over_direct": value / (st["rays_shot"] / td),
                                 "oracle_check": check}
        log(f"direct fp32: {pairs / td:.3e} pairs/s, {tf:.1f} TFLOP/s")

    plan.close()
    if not args.no_accuracy:
        result["accuracy_vs_rays"] = bench_accuracy(irs, synth, torch, stream)
    if not args.no_learned:
        result["learned"] = bench_learned(irs, synth, torch, stream, args, result)
    if not args.no_batch:
        result["batch"] = bench_batch(irs, synth, torch, stream)
    if not args.no_border:
        result["border"] = bench_border(irs, synth, torch, stream)
    if not args.no_circle:
        result["circle"] = bench_circle(irs, synth, torch, stream)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
