"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Sizes are ones the oracle finishes in seconds while spanning many ray tiles
(64 x 16 rays for the FP32 direct kernel, 64 x 4 for level 3) with ragged
edges in both directions, several level-1 cells and level-2 bands."""
import numpy as np
import pytest

import oracle as orc
import synth
from gpu_common import Case, check_map, rel_err, super_order

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def irs():
    import paper_2204_10871_amd as irs
    irs.load()
    return irs


def say(msg):
    print(msg, flush=True)


def _hist(px, npix):
    v = px[px >= 0]
    return np.bincount(v, minlength=npix * npix).astype(np.int64)


# ---------------------------------------------------------------------------
# direct sum, FP64
# ---------------------------------------------------------------------------
def test_direct_fp64_config1_full_map(irs):
    """The plain FP64 brute-force map (kappa_* = gamma = 0.3, S = 10, 256^2
    pixels, 2048^2 rays): every ray's alpha and pixel, and the map."""
    c = Case(0.3, 0.0, 0.3, 10.0, 256, n_rays=2048 ** 2, seed=synth.configs.CFG1.seed)
    say(f"cfg1 fp64: nx={c.geo.nx} ny={c.geo.ny} N*={c.lenses.n}")
    ref = c.oracle_direct()
    with c.plan("direct", "fp64") as pl:
        a1, a2, px = pl.deflect_grid(0, pl.n_rays)
        counts, st = pl.shoot_map()
    e = rel_err(a1, a2, ref["alpha1"], ref["alpha2"])
    assert e.max() < 1e-12, e.max()
    assert (px != ref["pix"]).sum() <= 2          # only exact pixel-edge ties may differ
    check_map(counts, ref["counts"], px, ref["pix"], min_agree=1 - 1e-6, max_rel_l1=1e-6)
    assert np.array_equal(_hist(px, 256), counts.ravel().astype(np.int64))
    assert st["rays_landed"] == int(counts.sum()) and st["rays_shot"] == pl.n_rays


@pytest.mark.parametrize("mass", ["unit", "salpeter"])
def test_direct_fp64_circular_plane(irs, mass):
    """The circular lens plane (Sec. 2.1, Eq. 9): lenses in the image
    rectangle's circumscribed circle, sheet -kappa_* theta; every ray and the
    map against the FP64 definition."""
    c = Case(0.3, 0.0, 0.3, 10.0, 256, n_rays=1024 ** 2, seed=synth.configs.CFG1.seed + 3,
             mass=mass, circle=True)
    say(f"circle fp64: nx={c.geo.nx} ny={c.geo.ny} N*={c.lenses.n} R={c.geo.lens_radius:.3f}")
    rect = Case(0.3, 0.0, 0.3, 10.0, 256, n_rays=1024 ** 2).geo.n_stars_expected     # 105
    assert c.lenses.n == c.geo.n_stars_expected > 2 * rect
    ref = c.oracle_direct()
    with c.plan("direct", "fp64") as pl:
        a1, a2, px = pl.deflect_grid(0, pl.n_rays)
        counts, st = pl.shoot_map()
    e = rel_err(a1, a2, ref["alpha1"], ref["alpha2"])
    assert e.max() < 1e-12, e.max()
    assert (px != ref["pix"]).sum() <= 2
    check_map(counts, ref["counts"], px, ref["pix"], min_agree=1 - 1e-5, max_rel_l1=1e-5)
    assert st["rays_landed"] == int(counts.sum())


# ---------------------------------------------------------------------------
# direct sum, FP32 with compensation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mass", ["unit", "salpeter"])
def test_direct_fp32_ragged(irs, mass):
    """Near-critical aspect (19:1) like the 4096^2 workloads, ~1000 lenses,
    a ray grid that is ragged against the 64 x 16 tiles in both directions."""
    c = Case(0.45, 0.05, 0.45, 5.0, 128, n_rays=1_000_003, mass=mass, seed=31)
    assert c.geo.nx % 64 and c.geo.ny % 16
    say(f"fp32 {mass}: nx={c.geo.nx} ny={c.geo.ny} N*={c.lenses.n}")
    ref = c.oracle_direct()
    with c.plan("direct", "fp32") as pl:
        a1, a2, px = pl.deflect_grid(0, pl.n_rays)
        counts, _ = pl.shoot_map()
    e = rel_err(a1, a2, ref["alpha1"], ref["alpha2"])
    say(f"  max e_r {e.max():.3e}  p99.99 {np.quantile(e, 0.9999):.3e}")
    assert np.mean(e <= 1e-5) >= 0.9999
    check_map(counts, ref["counts"], px, ref["pix"])
    assert np.array_equal(_hist(px, 128), counts.ravel().astype(np.int64))


def test_direct_fp32_large_plane(irs):
    """A plane ~370 theta_E long with N_* ~ 4500: the stars' mean field reaches
    ~80 theta_E at the ends, which FP32 only survives with compensation."""
    c = Case(0.45, 0.05, 0.45, 14.0, 256, n_rays=600_000, seed=32)
    say(f"fp32 large: ix={c.geo.ix:.1f} N*={c.lenses.n}")
    ids = np.arange(c.geo.n_rays)
    ref = c.oracle_direct()
    with c.plan("direct", "fp32") as pl:
        a1, a2, px = pl.deflect_grid(0, pl.n_rays)
    e = rel_err(a1, a2, ref["alpha1"], ref["alpha2"])
    say(f"  max e_r {e.max():.3e}")
    assert np.mean(e <= 1e-5) >= 0.9999
    assert np.mean(px == ref["pix"]) >= 0.9999
    del ids


# ---------------------------------------------------------------------------
# interpolation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["short_side", "l0_cells", "ray_multiple", "salpeter"])
def test_interp_matches_oracle(irs, kind):
    """GPU level-2/level-3 against the oracle's step-by-step interpolation
    (same approximation: agreement to rounding) and against the direct
    definition (the interpolation error budget)."""
    if kind == "short_side":
        c = Case(0.35, 0.1, 0.25, 4.0, 64, n_rays=400_000, seed=41)
    elif kind == "l0_cells":
        c = Case(0.35, 0.1, 0.25, 20.0, 96, n_rays=500_000, seed=42)
    elif kind == "ray_multiple":
        c = Case(0.45, 0.05, 0.45, 6.0, 128, n_rays=2_000_003, level2_ray_multiple=4.0, seed=43)
    else:
        c = Case(0.6, 0.0, 0.6, 12.0, 96, n_rays=500_000, mass="salpeter", seed=44)
    say(f"interp {kind}: n1={c.geo.n1x}x{c.geo.n1y} q={c.geo.q} N*={c.lenses.n}")
    ref2 = c.oracle_interp()
    ref1 = c.oracle_direct()
    with c.plan("interp", "fp64") as pl:
        assert pl.geometry["q"] == c.geo.q and pl.geometry["n1x"] == c.geo.n1x
        a1, a2, px = pl.deflect_grid(0, pl.n_rays)
        counts, _ = pl.shoot_map()
    e2 = rel_err(a1, a2, ref2["alpha1"], ref2["alpha2"])
    say(f"  vs O-2 max e_r {e2.max():.3e}")
    assert e2.max() < 1e-10
    assert np.mean(px == ref2["pix"]) >= 1 - 1e-5
    check_map(counts, ref2["counts"], px, ref2["pix"], min_agree=1 - 1e-5, max_rel_l1=1e-5)
    e1 = rel_err(a1, a2, ref1["alpha1"], ref1["alpha2"])
    say(f"  vs O-1 max e_r {e1.max():.3e}")
    assert np.mean(e1 <= 1e-4) >= 0.9999
    check_map(counts, ref1["counts"], px, ref1["pix"])
    assert np.array_equal(_hist(px, c.geo.npix), counts.ravel().astype(np.int64))


# ---------------------------------------------------------------------------
# edge cases and bookkeeping
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("offset", [0.0, 1e-7])
def test_interp_lenses_on_rays(irs, offset):
    """Lenses placed exactly on rays (rr = 0: their term is exactly zero) make
    the shared reciprocal of those rays' row groups fall back to one
    reciprocal per ray; lenses 1e-7 ray spacings off a ray (terms ~1e7 times
    the others in the group) go through the shared reciprocal.  Every ray
    still equals the oracle's interpolation to rounding."""
    c0 = Case(0.45, 0.05, 0.45, 5.0, 64, n_rays=300_000, seed=71)
    g0 = c0.geo
    rng = np.random.default_rng(72)
    ids = rng.choice(g0.nx * g0.ny, 40, replace=False)
    xs = g0.a1 + (ids % g0.nx + 0.5) * g0.ray_dx + offset * g0.ray_dx
    ys = g0.b1 + (ids // g0.nx + 0.5) * g0.ray_dy
    L = synth.Lenses(np.concatenate([c0.lenses.x, xs]), np.concatenate([c0.lenses.y, ys]), None)
    c = Case(0.45, 0.05, 0.45, 5.0, 64, n_rays=300_000, lenses=L)
    assert (c.geo.nx, c.geo.ny) == (g0.nx, g0.ny)
    ref = c.oracle_interp()
    with c.plan("interp", "fp64") as pl:
        a1, a2, px = pl.deflect_grid(0, pl.n_rays)
    e = rel_err(a1, a2, ref["alpha1"], ref["alpha2"])
    say(f"lenses {offset:g} spacings off rays: {L.n} lenses, max e_r vs O-2 {e.max():.3e}, "
        f"those rays {e[ids].max():.3e}")
    assert np.all(np.isfinite(a1)) and np.all(np.isfinite(a2))
    assert e.max() < 1e-10
    assert np.mean(px == ref["pix"]) >= 1 - 1e-5
def _ring_block_max(cs, n1x, n1y):
    """Most lenses in one block of 7 rows x 10 columns of level-1 cells: the
    ring lenses of four adjacent cells of a row (cell columns 4k .. 4k+3),
    which the level-2 points kernel stages in LDS when no block holds more
    than 768."""
    cnt = np.diff(np.asarray(cs, dtype=np.int64)).reshape(n1y, n1x)
    pre = np.zeros((n1y + 1, n1x + 1), np.int64)
    pre[1:, 1:] = cnt.cumsum(0).cumsum(1)
    best = 0
    for cy in range(n1y):
        ya, yb = max(0, cy - 3), min(n1y, cy + 4)
        for cx0 in range(0, n1x, 4):
            xa, xb = max(0, cx0 - 3), min(n1x, cx0 + 7)
            best = max(best, int(pre[yb, xb] - pre[ya, xb] - pre[yb, xa] + pre[ya, xa]))
    return best


@pytest.mark.parametrize("cluster", [0, 1200])
def test_interp_clustered_lenses(irs, cluster):
    """The level-2 points kernel reads the ring lenses (between a cell's 3 x 3
    and 7 x 7 blocks) from LDS when every four-cell workgroup's block of
    cells holds few enough of them, else from global memory.  A uniform
    field takes the first form; a cluster of 1200 lenses within a third of a
    cell side takes the second.  Both equal the oracle's interpolation to
    rounding."""
    c0 = Case(0.45, 0.05, 0.45, 6.0, 64, n_rays=300_000, seed=81)
    a1, a2, b1, b2 = c0.geo.rect
    rng = np.random.default_rng(82)
    side = np.sqrt((a2 - a1) * (b2 - b1) / (c0.lenses.n + cluster))   # level-1 side after
    r = side / 3 * np.sqrt(rng.random(cluster))
    t = 2 * np.pi * rng.random(cluster)
    xc, yc = a1 + 0.31 * (a2 - a1), b1 + 0.43 * (b2 - b1)
    L = synth.Lenses(np.concatenate([c0.lenses.x, xc + r * np.cos(t)]),
                     np.concatenate([c0.lenses.y, yc + r * np.sin(t)]), None)
    c = Case(0.45, 0.05, 0.45, 6.0, 64, n_rays=300_000, lenses=L)
    g = c.geo
    ref = c.oracle_interp()
    with c.plan("interp", "fp64") as pl:
        cs, _ = pl.level1()
        a1d, a2d, px = pl.deflect_grid(0, pl.n_rays)
        counts, _ = pl.shoot_map()
    most = _ring_block_max(cs, g.n1x, g.n1y)
    e = rel_err(a1d, a2d, ref["alpha1"], ref["alpha2"])
    say(f"cluster {cluster}: {L.n} lenses, cells {g.n1x}x{g.n1y}, most ring lenses of a "
        f"workgroup {most}, max e_r vs O-2 {e.max():.3e}")
    assert (most > 768) == (cluster > 0)
    assert e.max() < 1e-10
    assert np.mean(px == ref["pix"]) >= 1 - 1e-5
    check_map(counts, ref["counts"], px, ref["pix"], min_agree=1 - 1e-5, max_rel_l1=1e-5)


@pytest.mark.parametrize("method,precision", [("direct", "fp64"), ("direct", "fp32"),
                                              ("interp", "fp64")])
def test_star_free_map_exact(irs, method, precision):
    """No lenses: the map is the macro model's, identical to the oracle's."""
    empty = synth.Lenses(np.zeros(0), np.zeros(0), None)
    c = Case(0.0, 0.23, 0.11, 3.7, 37, n_rays=611 * 577, border=0.37, lenses=empty)
    ref = c.oracle_direct()
    with c.plan(method, precision) as pl:
        counts, st = pl.shoot_map()
        _, _, px = pl.deflect_grid(0, pl.n_rays, alpha=False)
    assert np.array_equal(px, ref["pix"])
    assert np.array_equal(counts.ravel(), ref["counts"])
    assert st["rays_landed"] == ref["landed"]


@pytest.mark.parametrize("method,precision", [("direct", "fp64"), ("direct", "fp32"),
                                              ("interp", "fp64")])
def test_single_ray_and_single_lens(irs, method, precision):
    """One ray (a 1 x 1 grid) and one lens off the ray, sheet off."""
    L = synth.Lenses(np.array([0.3]), np.array([-0.2]), None)
    c = Case(0.0, 0.0, 0.0, 2.0, 4, n_rays=1, border=1.0, sheet=False, lenses=L)
    assert c.geo.nx == 1 and c.geo.ny == 1
    ref = c.oracle_direct()
    with c.plan(method, precision) as pl:
        a1, a2, px = pl.deflect_grid(0, 1)
    e = rel_err(a1, a2, ref["alpha1"], ref["alpha2"])
    assert e.max() < (1e-12 if precision == "fp64" else 1e-6)
    assert px[0] == ref["pix"][0]


def test_each_map_computes_its_level2(irs):
    """irs_shoot_map computes every far-field expansion and coefficient band
    itself, also where the previous map left its whole band resident (this
    map fits one band), and gives the same map again."""
    c = Case(0.35, 0.1, 0.25, 4.0, 64, n_rays=400_000, seed=41)
    with c.plan("interp", "fp64") as pl:
        c1, s1 = pl.shoot_map(time_phases=True)
        c2, s2 = pl.shoot_map(time_phases=True)
    assert s1["level2_points"] > 0
    assert s2["level2_points"] == s1["level2_points"]
    assert s2["n_level2_launches"] == s1["n_level2_launches"] > 0
    assert np.array_equal(c1, c2)


@pytest.mark.parametrize("method,precision", [("direct", "fp32"), ("interp", "fp64")])
def test_row_bands_add_up_and_are_deterministic(irs, method, precision):
    """Disjoint row bands sum exactly to the full map (resume by bands), two
    runs are bitwise identical, and an unaligned ray range equals the same
    slice of a full per-ray evaluation."""
    c = Case(0.45, 0.05, 0.45, 5.0, 96, n_rays=300_007, seed=51)
    with c.plan(method, precision) as pl:
        full, _ = pl.shoot_map()
        again, _ = pl.shoot_map()
        assert np.array_equal(full, again)
        ny = pl.geometry["ny"]
        acc = np.zeros(96 * 96, np.uint32)
        cuts = [0, 7, ny // 3, ny // 3 + 1, ny - 5, ny]
        for r0, r1 in zip(cuts[:-1], cuts[1:]):
            pl.shoot_rows(r0, r1 - r0, acc)
        assert np.array_equal(acc.reshape(96, 96), full)
        a1, a2, px = pl.deflect_grid(0, pl.n_rays)
        first, n = 12345, 54321
        b1, b2, qx = pl.deflect_grid(first, n)
        assert np.array_equal(b1, a1[first:first + n]) and np.array_equal(qx, px[first:first + n])


def test_critical_and_invalid_plans(irs):
    p = irs.make_params(0.5, 0.0, 0.5, 100.0, 64, rays_per_pixel=10.0)
    with pytest.raises(irs.IrsError) as e:
        irs.Plan(p, np.zeros(3), np.zeros(3))
    assert e.value.status == 2
    c = Case(0.3, 0.0, 0.3, 3.0, 16, n_rays=10_000, seed=3)
    with c.plan("direct", "fp64") as pl:
        with pytest.raises(irs.IrsError):
            pl.deflect_grid(pl.n_rays - 5, 10)
        with pytest.raises(irs.IrsError):
            pl.shoot_rows(-1, 3, np.zeros(16 * 16, np.uint32))


@pytest.mark.parametrize("draw", [3, 4, 6])
def test_tree_sides_on_batch_maps_equal_paper_form(irs, draw):
    """Maps of the 64-map batch (2477, 25176 and 9115 lenses): the sides the
    plan picks for its distant-field tree tile their parents by workgroups,
    and the deflections equal those of the paper's per-point sums, on coarse
    level-2 grids (q = 4)."""
    import paper_2204_10871_amd as irs_mod
    d = synth.configs.batch_draws()[draw]
    S = irs_mod.source_side_for_n_star(d.kappa_star, d.kappa_c, d.gamma, d.n_star_target)
    c = Case(d.kappa_star, d.kappa_c, d.gamma, S, 256, n_rays=16 * 16 * d.n_star_target,
             level2_ray_multiple=4.0, n_lens=d.n_star_target, seed=d.seed)
    assert c.geo.q == 4
    L = c.lenses
    out = {}
    for paper in (False, True):
        p = irs_mod.make_params(**c.kw, method="interp", precision="fp64",
                                level2_paper=paper, **c.p_extra)
        with irs_mod.Plan(p, L.x, L.y, L.m) as pl:
            a1, a2, px = pl.deflect_grid(0, pl.n_rays)
            counts, st = pl.shoot_map()
        out[paper] = (a1, a2, px, counts, st)
    st = out[False][4]
    say(f"batch map {draw}: N*={L.n} cells {c.geo.n1x}x{c.geo.n1y}, super {st['super_cells']}, "
        f"mid {st['mid_cells']}")
    if st["mid_cells"] > 0:
        assert st["super_cells"] % (4 * st["mid_cells"]) == 0
    e = rel_err(out[False][0], out[False][1], out[True][0], out[True][1])
    say(f"  max e_r tree vs paper form {e.max():.3e}")
    assert e.max() < 1e-11
    assert np.mean(out[False][2] == out[True][2]) >= 1 - 1e-6


def test_three_level_field_equals_paper_form(irs):
    """At 3e4 lenses the distant field goes through super cells, mid cells and
    the cells themselves; the deflections it gives equal those of the
    per-point sums over every distant lens (the paper's form) to FP64
    rounding, on a coarse level-2 grid (q = 4) that keeps the latter cheap."""
    import paper_2204_10871_amd as irs_mod
    S = irs_mod.source_side_for_n_star(0.45, 0.05, 0.45, 30000)
    c = Case(0.45, 0.05, 0.45, S, 256, n_rays=2_000_000, level2_ray_multiple=2.0,
             n_lens=30000, seed=63)
    g = c.geo
    assert g.q == 4
    assert super_order(g) == 40        # the 40-term super and mid instances
    L = c.lenses
    out = {}
    for paper in (False, True):
        p = irs_mod.make_params(**c.kw, method="interp", precision="fp64",
                                level2_paper=paper, **c.p_extra)
        with irs_mod.Plan(p, L.x, L.y, L.m) as pl:
            a1, a2, px = pl.deflect_grid(0, pl.n_rays)
            counts, st = pl.shoot_map()
        out[paper] = (a1, a2, px, counts, st)
    st = out[False][4]
    say(f"three levels: cells {g.n1x}x{g.n1y}, super {st['super_cells']}, mid {st['mid_cells']}")
    assert st["super_cells"] > st["mid_cells"] > 0
    assert out[True][4]["super_cells"] == 0
    e = rel_err(out[False][0], out[False][1], out[True][0], out[True][1])
    say(f"  max e_r three-level vs paper form {e.max():.3e}")
    assert e.max() < 1e-11
    assert np.mean(out[False][2] == out[True][2]) >= 1 - 1e-6
    assert np.abs(out[False][3].astype(np.int64) - out[True][3]).sum() <= 2 * np.sum(out[False][2] != out[True][2])


@pytest.mark.parametrize("kind", ["square_cells", "oblong_cells"])
def test_level2_local_expansion_equals_paper_form(irs, kind):
    """The per-cell local expansion gives the same level-2 coefficients as the
    per-point sum over all distant lenses (the paper's form), to FP64 rounding:
    identical per-ray deflections to 1e-11 and identical maps."""
    if kind == "square_cells":
        c = Case(0.6, 0.0, 0.6, 14.0, 96, n_rays=400_000, mass="salpeter", seed=61)
    else:   # I_y/dx1 just above 10: 191 x 11 cells of aspect ~1.1 (expansion order 48)
        c = Case(0.45, 0.05, 0.45, 11.75, 64, n_rays=300_000, seed=62)
    g = c.geo
    say(f"level-2 forms {kind}: cells {g.n1x}x{g.n1y} w1={g.ix / g.n1x:.3f} h1={g.iy / g.n1y:.3f}")
    # super and mid series: 40 terms for square cells, 48 for these oblong ones
    assert super_order(g) == (40 if kind == "square_cells" else 48)
    import paper_2204_10871_amd as irs_mod
    L = c.lenses
    out = {}
    for paper in (False, True):
        p = irs_mod.make_params(**c.kw, method="interp", precision="fp64",
                                level2_paper=paper, **c.p_extra)
        with irs_mod.Plan(p, L.x, L.y, L.m) as pl:
            a1, a2, px = pl.deflect_grid(0, pl.n_rays)
            counts, st = pl.shoot_map()
        out[paper] = (a1, a2, px, counts)
    e = rel_err(out[False][0], out[False][1], out[True][0], out[True][1])
    say(f"  max e_r local vs paper form {e.max():.3e}")
    assert e.max() < 1e-11
    assert np.mean(out[False][2] == out[True][2]) >= 1 - 1e-6
    assert np.abs(out[False][3].astype(np.int64) - out[True][3]).sum() <= 2 * np.sum(out[False][2] != out[True][2])


def test_single_ray_calls_equal_row_calls(irs):
    """Tiles follow the level-1 cells where cells are wide, so a cell's last
    column tile is narrower than a wave and its spare lanes hold the next
    cell's first columns; a call for one ray must still take that ray from
    its own tile.  Rays at both edges of every level-1 column, shot one at a
    time, equal the same rays of whole-row calls bit for bit."""
    c = Case(0.35, 0.1, 0.25, 20.0, 96, n_rays=8_000_000, seed=46)
    with c.plan("interp", "fp64") as pl:
        g = pl.geometry
        assert g["nx"] // g["n1x"] >= 96            # columns per cell: tiles follow cells
        rows = [0, g["ny"] // 3, g["ny"] - 1]
        for j in rows:
            ra1, ra2, rpx = pl.deflect_grid(j * g["nx"], g["nx"])
            cols = []
            for cx in range(g["n1x"]):
                i0, i1 = pl.level1_col_rays(cx)
                cols += [i0, i0 + 1, i0 + 3, i1 - 4, i1 - 1]
            for i in cols:
                a1, a2, px = pl.deflect_grid(j * g["nx"] + i, 1)
                assert (a1[0], a2[0], px[0]) == (ra1[i], ra2[i], rpx[i]), (j, i)


def _clustered_lenses(rect, n, n_pile, seed):
    """n lenses uniform over rect, of which n_pile (spread through the input
    order) sit inside a square of side 2e-4 well inside one level-1 cell."""
    L = synth.uniform_lenses(n, rect, seed)
    x, y = L.x.copy(), L.y.copy()
    cx = rect[0] + 0.3137 * (rect[1] - rect[0])
    cy = rect[2] + 0.6071 * (rect[3] - rect[2])
    idx = np.arange(0, n, n // n_pile)[:n_pile]
    u = synth.uniform_lenses(n_pile, (-1e-4, 1e-4, -1e-4, 1e-4), seed + 1)
    x[idx] = cx + u.x
    y[idx] = cy + u.y
    return synth.Lenses(x, y, None)


def _edge_lenses(geo, n, seed):
    """Lenses on level-1 cell edges (and the rect's own edges) and uniform ones."""
    L = synth.uniform_lenses(n, geo.rect, seed)
    x, y = L.x.copy(), L.y.copy()
    w1 = (geo.rect[1] - geo.rect[0]) / geo.n1x
    h1 = (geo.rect[3] - geo.rect[2]) / geo.n1y
    k = np.arange(n // 2)
    x[: n // 2] = geo.rect[0] + (k % (geo.n1x + 1)) * w1
    y[: n // 2] = geo.rect[2] + (k % (geo.n1y + 1)) * h1
    return synth.Lenses(np.minimum(x, geo.rect[1]), np.minimum(y, geo.rect[3]), None)


@pytest.mark.parametrize("kind", ["uniform_ragged", "clustered", "cell_edges", "one_lens"])
def test_level1_packing_equals_oracle(irs, kind):
    """The packing (Sec. 2.4 flow chart, lenses into level-1 cells) equals the
    oracle's stable counting sort index for index: same cell_start, and inside
    every cell the lenses in input order.  "clustered" puts a third of the
    lenses into one cell, "uniform_ragged" needs three 8-bit digit passes
    (about 1e5 cells) with a lens count that is no multiple of the 1024-lens
    sort block."""
    kw = (0.45, 0.05, 0.45, 25.0, 64)
    g0 = Case(*kw, n_rays=10_000, n_lens=8).geo
    if kind == "uniform_ragged":
        c = Case(*kw, n_rays=10_000, n_lens=100_003, seed=51)
    elif kind == "clustered":
        c = Case(*kw, n_rays=10_000, lenses=_clustered_lenses(g0.rect, 90_000, 30_000, 52))
    elif kind == "cell_edges":
        g1 = Case(*kw, n_rays=10_000, n_lens=20_000).geo
        c = Case(*kw, n_rays=10_000, lenses=_edge_lenses(g1, 20_000, 53))
        assert (c.geo.n1x, c.geo.n1y) == (g1.n1x, g1.n1y)
    else:
        c = Case(*kw, n_rays=10_000, lenses=synth.Lenses(np.array([1.5]), np.array([-2.0]), None))
    ncell = c.geo.n1x * c.geo.n1y
    say(f"level1 {kind}: N*={c.lenses.n} cells={ncell}")
    cs_ref, perm_ref = orc.level1(c.geo, c.lenses)
    with c.plan("interp", "fp64") as pl:
        cs, order = pl.level1()
    assert np.array_equal(cs.astype(np.int64), cs_ref)
    assert np.array_equal(order.astype(np.int64), perm_ref)
    if kind == "clustered":
        assert np.diff(cs_ref).max() >= 30_000
    if kind == "uniform_ragged":
        assert ncell > 1 << 16
