"""Pins of the oracle's interpolation (O-2: level-1 packing, level-2 far-field
Taylor coefficients with the sheet, level-3 evaluation) against mathematics
independent of its code paths: the partition property, the exact Taylor
remainder of 1/(z - z_i), agreement with the direct definition at h = 0,
the convergence order in the level-2 spacing and 50-digit brute force."""
import numpy as np
import pytest

import synth


def _small(orc, sheet=True, n_lens=None, level2_spacing=None, mass="salpeter", seed=11):
    g0 = orc.geometry(0.35, 0.1, 0.25, 4.0, 48, n_rays=260 * 190, sheet=sheet,
                      level2_spacing=level2_spacing)
    n = g0.n_stars_expected if n_lens is None else n_lens
    g = g0.with_lens_count(n)
    L = synth.uniform_lenses(n, g.rect, seed, mass=mass)
    return g, L


def _cells_numpy(g, L):
    w1, h1 = (g.a2 - g.a1) / g.n1x, (g.b2 - g.b1) / g.n1y
    cx = np.clip(np.floor((L.x - g.a1) / w1).astype(np.int64), 0, g.n1x - 1)
    cy = np.clip(np.floor((L.y - g.b1) / h1).astype(np.int64), 0, g.n1y - 1)
    return cx, cy


def test_level1_partition(orc):
    g, L = _small(orc)
    cs, perm = orc.level1(g, L)
    assert cs[0] == 0 and cs[-1] == L.n and np.all(np.diff(cs) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(L.n))
    cx, cy = _cells_numpy(g, L)
    cell = cy * g.n1x + cx
    for c in range(g.n1x * g.n1y):
        members = perm[cs[c]:cs[c + 1]]
        assert np.array_equal(members, np.flatnonzero(cell == c))


def _near_sum(g, L, z, cx, cy):
    lcx, lcy = _cells_numpy(g, L)
    near = (np.abs(lcx - cx) <= 1) & (np.abs(lcy - cy) <= 1)
    d = z - (L.x[near] + 1j * L.y[near])
    m = L.masses()[near]
    return np.sum(m * d / np.abs(d) ** 2)     # alpha1 + i alpha2 of the near lenses


def _level2_xy(g, gx, gy):
    w2, h2 = (g.a2 - g.a1) / (g.n1x * g.q), (g.b2 - g.b1) / (g.n1y * g.q)
    return g.a1 + (gx + 0.5) * w2, g.b1 + (gy + 0.5) * h2


def test_h0_matches_direct(orc):
    """At a level-2 point itself (h = 0): conj(C0) + near lenses + macro term
    equals the direct definition (O-1) there; in the four corner cells C0
    carries no sheet and the closed-form sheet is added instead."""
    g, L = _small(orc)
    cs, perm = orc.level1(g, L)
    rng = np.random.default_rng(5)
    nx2, ny2 = g.n1x * g.q, g.n1y * g.q
    gx = np.concatenate([rng.integers(0, nx2, 40), [0, nx2 - 1, 0, nx2 - 1]])
    gy = np.concatenate([rng.integers(0, ny2, 40), [0, 0, ny2 - 1, ny2 - 1]])
    C = orc.level2(g, L, cs, perm, gx, gy)
    x, y = _level2_xy(g, gx, gy)
    ax, ay, _ = orc.alpha_points(g, L, x, y)
    for k in range(gx.size):
        cx, cy = gx[k] // g.q, gy[k] // g.q
        z = x[k] + 1j * y[k]
        got = np.conj(C[k, 0]) + _near_sum(g, L, z, cx, cy) \
            + (g.kappa + g.gamma) * x[k] + 1j * (g.kappa - g.gamma) * y[k]
        corner = cx in (0, g.n1x - 1) and cy in (0, g.n1y - 1)
        if corner:
            I1, I2 = orc.sheet_I(g.rect, [x[k]], [y[k]])
            got += -(g.kappa_star / np.pi) * (I1[0] + 1j * I2[0])
        want = ax[k] + 1j * ay[k]
        assert abs(got - want) < 1e-11 * max(1.0, abs(want))


def _far_remainder(g, L, ray_ids):
    """Exact remainder of the order-4 far expansion: for each ray,
    sum_far m_i (-h)^5 / ((z0 - z_i)^5 (z - z_i))  (conjugated deflection)."""
    lcx, lcy = _cells_numpy(g, L)
    out = np.empty(ray_ids.size, complex)
    for k, r in enumerate(ray_ids):
        i, j = r % g.nx, r // g.nx
        z = (g.a1 + (i + 0.5) * g.ray_dx) + 1j * (g.b1 + (j + 0.5) * g.ray_dy)
        gx = ((2 * i + 1) * g.n1x * g.q) // (2 * g.nx)
        gy = ((2 * j + 1) * g.n1y * g.q) // (2 * g.ny)
        x0, y0 = _level2_xy(g, gx, gy)
        z0 = x0 + 1j * y0
        cx, cy = gx // g.q, gy // g.q
        far = ~((np.abs(lcx - cx) <= 1) & (np.abs(lcy - cy) <= 1))
        zi = L.x[far] + 1j * L.y[far]
        h = z - z0
        out[k] = np.sum(L.masses()[far] * (-h) ** 5 / ((z0 - zi) ** 5 * (z - zi)))
    return out


def test_far_remainder_identity(orc):
    """Without the sheet: alpha_interp - alpha_direct is exactly minus the
    conjugate of the order-5 Taylor remainder of the distant lenses (exact algebra:
    1/(w+h) - sum_{k<5} (-h)^k/w^(k+1) = (-h)^5/(w^5 (w+h))).  A wrong C_k for
    any k, a wrong near/far split or a wrong level-2 point breaks it."""
    g, L = _small(orc, sheet=False)
    cs, perm = orc.level1(g, L)
    coef = orc.level2_grid(g, L, cs, perm, threads=8)
    rng = np.random.default_rng(8)
    ids = rng.choice(g.n_rays, 300, replace=False)
    it = orc.shoot_interp(g, L, cs, perm, coef, ray_ids=ids)
    dr = orc.shoot_direct(g, L, ray_ids=ids)
    diff = (it["alpha1"] - dr["alpha1"]) + 1j * (it["alpha2"] - dr["alpha2"])
    want = -np.conj(_far_remainder(g, L, ids))
    scale = np.maximum(1.0, np.hypot(dr["alpha1"], dr["alpha2"]))
    assert np.all(np.abs(diff - want) < 1e-11 * scale)
    assert np.max(np.abs(want)) > 1e-12      # the identity is not vacuous


def test_sheet_in_interpolation_matches_closed_form(orc):
    """With the sheet: alpha_interp - alpha_direct = -conj(far remainder)
    - kappa_* conj(F_series(z) - F(z)), where F is the closed form; the sheet
    part is the series' own O(h^5) remainder, small at these spacings."""
    g, L = _small(orc, sheet=True)
    cs, perm = orc.level1(g, L)
    coef = orc.level2_grid(g, L, cs, perm, threads=8)
    rng = np.random.default_rng(9)
    ids = rng.choice(g.n_rays, 200, replace=False)
    it = orc.shoot_interp(g, L, cs, perm, coef, ray_ids=ids)
    dr = orc.shoot_direct(g, L, ray_ids=ids)
    diff = (it["alpha1"] - dr["alpha1"]) + 1j * (it["alpha2"] - dr["alpha2"])
    far = -np.conj(_far_remainder(g, L, ids))
    scale = np.maximum(1.0, np.hypot(dr["alpha1"], dr["alpha2"]))
    # the remaining difference is the sheet series' own O(h^5) remainder
    resid = np.abs(diff - far)
    assert np.all(resid < 1e-9 * scale), resid.max()


def test_convergence_in_level2_spacing(orc):
    """Halving the level-2 spacing shrinks the interpolation error by ~2^5."""
    errs = []
    for dx2 in (0.16, 0.08):
        g, L = _small(orc, sheet=False, level2_spacing=dx2, mass="unit", seed=21)
        cs, perm = orc.level1(g, L)
        coef = orc.level2_grid(g, L, cs, perm, threads=8)
        ids = np.random.default_rng(2).choice(g.n_rays, 400, replace=False)
        it = orc.shoot_interp(g, L, cs, perm, coef, ray_ids=ids)
        dr = orc.shoot_direct(g, L, ray_ids=ids)
        errs.append(np.sqrt(np.mean((it["alpha1"] - dr["alpha1"]) ** 2
                                    + (it["alpha2"] - dr["alpha2"]) ** 2)))
    ratio = errs[0] / errs[1]
    assert 16 < ratio < 64, (errs, ratio)


def test_level2_brute_force_50_digits(orc):
    """C_0..C_4 of the distant lenses (no sheet) at a few points against
    50-digit sums of m (-1)^k / (z0 - z_i)^(k+1)."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    g, L = _small(orc, sheet=False)
    cs, perm = orc.level1(g, L)
    gx = np.array([3, 57, 140])
    gy = np.array([2, 33, 70])
    gx = np.minimum(gx, g.n1x * g.q - 1)
    gy = np.minimum(gy, g.n1y * g.q - 1)
    C = orc.level2(g, L, cs, perm, gx, gy)
    lcx, lcy = _cells_numpy(g, L)
    x, y = _level2_xy(g, gx, gy)
    for k in range(gx.size):
        cx, cy = gx[k] // g.q, gy[k] // g.q
        z0 = mpmath.mpc(x[k], y[k])
        acc = [mpmath.mpc(0)] * 5
        for i in range(L.n):
            if abs(lcx[i] - cx) <= 1 and abs(lcy[i] - cy) <= 1:
                continue
            w = z0 - mpmath.mpc(L.x[i], L.y[i])
            for j in range(5):
                acc[j] += mpmath.mpf(L.m[i]) * (-1) ** j / w ** (j + 1)
        for j in range(5):
            ref = complex(acc[j])
            assert abs(C[k, j] - ref) <= 1e-12 * max(abs(ref), 1e-3)


@pytest.mark.parametrize("sheet,mass", [(True, "salpeter"), (False, "unit")])
def test_per_ray_level2_equals_grid(orc, sheet, mass):
    """O-2 with each ray's own level-2 point summed on the spot equals O-2 with
    the whole level-2 grid, bit for bit, on rays spread over the map with the
    four corner cells and the edge rows and columns included; and the per-ray
    form obeys the exact far-remainder identity by itself (no sheet)."""
    g, L = _small(orc, sheet=sheet, mass=mass, seed=31)
    cs, perm = orc.level1(g, L)
    coef = orc.level2_grid(g, L, cs, perm, threads=8)
    rng = np.random.default_rng(12)
    nx, ny = g.nx, g.ny
    corners = [0, nx - 1, (ny - 1) * nx, ny * nx - 1]
    edges = list(rng.integers(0, nx, 20)) + list((ny - 1) * nx + rng.integers(0, nx, 20)) \
        + list(rng.integers(0, ny, 20) * nx) + list(rng.integers(0, ny, 20) * nx + nx - 1)
    ids = np.unique(np.concatenate([rng.choice(g.n_rays, 300, replace=False), corners, edges]))
    grid = orc.shoot_interp(g, L, cs, perm, coef, ray_ids=ids, want_counts=True)
    own = orc.shoot_interp_rays(g, L, cs, perm, ray_ids=ids, want_counts=True, threads=8)
    for k in ("alpha1", "alpha2", "pix", "counts"):
        assert np.array_equal(grid[k], own[k]), k
    assert (grid["landed"], grid["off"]) == (own["landed"], own["off"])
    rng_r = orc.shoot_interp_rays(g, L, cs, perm, first=5 * nx + 3, n=700, threads=2)
    rng_g = orc.shoot_interp(g, L, cs, perm, coef, first=5 * nx + 3, n=700)
    assert np.array_equal(rng_r["alpha1"], rng_g["alpha1"])
    if not sheet:
        dr = orc.shoot_direct(g, L, ray_ids=ids)
        diff = (own["alpha1"] - dr["alpha1"]) + 1j * (own["alpha2"] - dr["alpha2"])
        want = -np.conj(_far_remainder(g, L, ids))
        scale = np.maximum(1.0, np.hypot(dr["alpha1"], dr["alpha2"]))
        assert np.all(np.abs(diff - want) < 1e-11 * scale)
