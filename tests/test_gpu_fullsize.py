"""Full-size parity: the benchmark workloads at their real sizes, in the launch
configuration the benchmark times (one band of ray rows per call), checked on
outputs the oracle can compute one by one, and by properties that hold at any
size (the band's map is the histogram of its per-ray pixels, bit for bit)."""
import numpy as np
import pytest

import oracle as orc
import synth
from gpu_common import THREADS, rel_err

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def irs():
    import paper_2204_10871_amd as irs
    irs.load()
    return irs


def _workload(irs, w, method, precision, **over):
    p = irs.params_from_workload(w, method=method, precision=precision, **over)
    g0 = irs.geometry(p, 0)
    n = g0["n_stars_expected"]
    L = synth.uniform_lenses(n, (g0["a1"], g0["a2"], g0["b1"], g0["b2"]), w.seed, mass=w.mass,
                             m_min=w.m_min, m_max=w.m_max)
    og = orc.geometry(w.kappa_star, w.kappa_c, w.gamma, w.source_side, w.npix,
                      rays_per_pixel=w.rays_per_pixel, n_rays=w.n_rays, n_lens=n,
                      level2_ray_multiple=w.level2_ray_multiple or None)
    return p, L, og


def _band_check(irs, pl, j0, j1, og, L, n_sample, tol_e, seed=5):
    """Whole band on the device: per-ray pixels vs the band's map (exact), and
    a sample of rays vs the oracle's direct definition."""
    import torch
    nx = pl.geometry["nx"]
    npix = pl.params.npix_side
    n = (j1 - j0) * nx
    px = torch.empty(n, dtype=torch.int64, device="cuda:0")
    a1d = torch.empty(n, dtype=torch.float64, device="cuda:0")
    a2d = torch.empty(n, dtype=torch.float64, device="cuda:0")
    pl.deflect_grid_device(j0 * nx, n, a1d, a2d, px)
    counts = torch.zeros(npix * npix, dtype=torch.int32, device="cuda:0")
    st = pl.shoot_rows(j0, j1 - j0, counts)
    torch.cuda.synchronize()
    hist = torch.bincount(px[px >= 0], minlength=npix * npix).to(torch.int32)
    assert torch.equal(hist, counts), "band map != histogram of its per-ray pixels"
    assert st["rays_landed"] == int((px >= 0).sum().item())
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(n, n_sample, replace=False)) + j0 * nx
    ref = orc.shoot_direct(og, L, ray_ids=ids, threads=THREADS, want_counts=False)
    sel = torch.as_tensor(ids - j0 * nx, device="cuda:0")
    gpx = px[sel].cpu().numpy()
    a1 = a1d[sel].cpu().numpy()
    a2 = a2d[sel].cpu().numpy()
    del px, a1d, a2d
    e = rel_err(a1, a2, ref["alpha1"], ref["alpha2"])
    mism = int(np.sum(gpx != ref["pix"]))
    say(f"  band rows {j0}..{j1}: {n:.3e} rays, sample {n_sample}: max e_r {e.max():.2e}, "
        f"pixel mismatches {mism}")
    assert np.sum(e > tol_e) <= n_sample // 10000
    assert mism <= max(1, n_sample // 10000)


def test_1e6_lens_map_interp_band(irs):
    """kappa_* = gamma = 0.6, 1e6 Salpeter lenses, 10000^2 px, 1000 rays/px:
    one level-1 row band (2.2e8 rays), interpolated path as benchmarked."""
    w = synth.configs.CFG3
    p, L, og = _workload(irs, w, "interp", "fp64")
    with irs.Plan(p, L.x, L.y, L.m) as pl:
        say(f"1e6-lens map: {pl.geometry['nx']}x{pl.geometry['ny']} rays, N*={L.n}")
        j0, j1 = pl.level1_row_rays(pl.geometry["n1y"] // 2 + 3)
        _band_check(irs, pl, j0, j1, og, L, 1500, 1e-4)
        j0, j1 = pl.level1_row_rays(1)          # near the rectangle's edge
        _band_check(irs, pl, j0, j1, og, L, 500, 1e-4, seed=6)


def test_1e6_lens_map_direct_fp32_strip(irs):
    """The FP32 direct sum at N_* = 1e6 on the same map: a 16-row strip."""
    w = synth.configs.CFG3
    p, L, og = _workload(irs, w, "direct", "fp32")
    with irs.Plan(p, L.x, L.y, L.m) as pl:
        j0 = pl.geometry["ny"] // 2 // 16 * 16 + 32
        _band_check(irs, pl, j0, j0 + 16, og, L, 1500, 1e-5)


@pytest.mark.parametrize("which", ["s25", "n1e5"])
def test_4096_map_bands(irs, which):
    """kappa_* = gamma = 0.45, kappa_c = 0.05 (aspect 19), 4096^2 px, 100
    rays/px, coarse grid at 16 ray spacings: S = 25 (4450 lenses) and the
    1e5-lens variant; interpolated band and FP32 direct strip."""
    w = synth.configs.CFG2 if which == "s25" else synth.configs.CFG2T
    for method, precision, tol in (("interp", "fp64", 1e-4), ("direct", "fp32", 1e-5)):
        p, L, og = _workload(irs, w, method, precision)
        with irs.Plan(p, L.x, L.y, L.m) as pl:
            say(f"4096^2 {which} {method}: {pl.geometry['nx']}x{pl.geometry['ny']} rays, "
                f"N*={L.n}, q={pl.geometry['q']}")
            if method == "interp":
                j0, j1 = pl.level1_row_rays(pl.geometry["n1y"] // 2)
            else:
                j0 = pl.geometry["ny"] // 2 // 16 * 16
                j1 = j0 + 16
            _band_check(irs, pl, j0, j1, og, L, 1500, tol)


def test_1e6_lens_learned_band(irs):
    """The learned interpolant at its full-size workload (kappa_* = gamma = 0.5,
    kappa_c = 0.05, 1e6 unit lenses, 8192^2 px, 100 rays/px): trained with the
    default settings, then one level-1 row band checked as above."""
    w = synth.configs.CFG5
    p, L, og = _workload(irs, w, "learned", "fp64")
    with irs.Plan(p, L.x, L.y, L.m) as pl:
        rep = pl.learn(synth.network.fourier_frequencies(7), irs.learn_params())
        say(f"learned 1e6: val mean {rep['val_mean_abs']:.2e} (grid alone {rep['base_mean_abs']:.2e},"
            f" tol {rep['tol_mean']:.2e}), p99.99 {rep['val_p9999_abs']:.2e}, "
            f"fallback {rep['fallback']}, train {rep['ms_train']:.0f} ms")
        assert rep["fallback"] == 0
        j0, j1 = pl.level1_row_rays(pl.geometry["n1y"] // 2 + 1)
        _band_check(irs, pl, j0, j1, og, L, 1500, 1e-4)


def _spread_ray_ids(pl, rng, n_random, per_edge):
    """Ray ids over the whole map: n_random uniform draws over every ray index,
    plus per_edge draws in each of the first and last level-1 rows and columns
    (the edge bands) and per_edge // 4 in each of the four corner level-1
    cells.  Sorted and unique."""
    g = pl.geometry
    nx, ny = g["nx"], g["ny"]
    rows = [pl.level1_row_rays(c) for c in (0, g["n1y"] - 1)]
    cols = [pl.level1_col_rays(c) for c in (0, g["n1x"] - 1)]
    ids = [rng.choice(nx * ny, n_random, replace=False)]
    for j0, j1 in rows:
        ids.append(rng.integers(j0, j1, per_edge) * nx + rng.integers(0, nx, per_edge))
    for i0, i1 in cols:
        ids.append(rng.integers(0, ny, per_edge) * nx + rng.integers(i0, i1, per_edge))
    for j0, j1 in rows:
        for i0, i1 in cols:
            k = max(1, per_edge // 4)
            ids.append(rng.integers(j0, j1, k) * nx + rng.integers(i0, i1, k))
    return np.unique(np.concatenate(ids))


def _gpu_rays(pl, ids):
    """alpha and pixel of listed rays, one irs_deflect_grid call per ray (in
    ray order, so each level-2 band is computed once)."""
    a1 = np.empty(ids.size)
    a2 = np.empty(ids.size)
    px = np.empty(ids.size, np.int64)
    for k, r in enumerate(ids):
        x1, x2, p = pl.deflect_grid(int(r), 1)
        a1[k], a2[k], px[k] = x1[0], x2[0], p[0]
    return a1, a2, px


@pytest.mark.timeout(900)
@pytest.mark.parametrize("which", ["n1e6_salpeter", "n1e5_4096"])
def test_three_level_field_vs_per_ray_oracle(irs, which):
    """The distant field at full size (super, mid and cell expansions active)
    against the oracle's interpolation with each ray's own level-2 point summed
    over every distant lens (O-2 per ray, Sec. 2.4 level-2 coefficients): both
    evaluate the same fourth-order series, so they agree to FP64 rounding.
    Rays spread over the whole map, the edge bands and the corner cells
    included; also against the direct definition at the interpolation budget."""
    w = synth.configs.CFG3 if which == "n1e6_salpeter" else synth.configs.CFG2T
    p, L, og = _workload(irs, w, "interp", "fp64")
    with irs.Plan(p, L.x, L.y, L.m) as pl:
        rng = np.random.default_rng(17)
        n_rand, per_edge = (1200, 200) if which == "n1e6_salpeter" else (1600, 200)
        ids = _spread_ray_ids(pl, rng, n_rand, per_edge)
        say(f"{which}: {pl.geometry['nx']}x{pl.geometry['ny']} rays, N*={L.n}, "
            f"level-1 {pl.geometry['n1x']}x{pl.geometry['n1y']}, q={pl.geometry['q']}, "
            f"{ids.size} rays")
        a1, a2, px = _gpu_rays(pl, ids)
        import torch
        counts = torch.zeros(w.npix * w.npix, dtype=torch.int32, device="cuda:0")
        sides = pl.shoot_rows(0, 1, counts)       # reports the tree's cell sides
        del counts
    assert sides["super_cells"] > 0, "the distant-field tree is not active"
    cs, perm = orc.level1(og, L)
    ref = orc.shoot_interp_rays(og, L, cs, perm, ray_ids=ids, threads=THREADS)
    d = np.hypot(a1 - ref["alpha1"], a2 - ref["alpha2"])
    e = d / np.maximum(np.hypot(ref["alpha1"], ref["alpha2"]), 1.0)
    mism = int(np.sum(px != ref["pix"]))
    say(f"  tree (K_S={sides['super_cells']}, K_M={sides['mid_cells']}) vs per-ray O-2: "
        f"max |d alpha| {d.max():.2e}, max e_r {e.max():.2e}, pixel mismatches {mism}")
    assert d.max() < 1e-10, d.max()
    assert mism == 0
    ref1 = orc.shoot_direct(og, L, ray_ids=ids, threads=THREADS, want_counts=False)
    e1 = rel_err(a1, a2, ref1["alpha1"], ref1["alpha2"])
    mis1 = int(np.sum(px != ref1["pix"]))
    say(f"  vs O-1: max e_r {e1.max():.2e}, pixel mismatches {mis1}")
    assert np.sum(e1 > 1e-4) <= ids.size // 10000
    assert mis1 <= max(1, ids.size // 10000)
