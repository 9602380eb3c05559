"""Oracle geometry against the printed sizing rules and invariants, and the
seeded input generator against its distributions."""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_border_and_rectangle(orc):
    fig8 = GOLDEN["fig8_setup"]
    g = orc.geometry(fig8["kappa_star"], fig8["kappa"] - fig8["kappa_star"], fig8["gamma"],
                     fig8["source_side"], fig8["npix"], rays_per_pixel=fig8["rays_per_pixel"])
    P = GOLDEN["border_factor"]["value"] * math.sqrt(fig8["kappa_star"])
    assert g.border == pytest.approx(P)
    # gamma = 0: the rectangle is a square of side (S + 2P)/|1 - kappa|
    assert g.ix == pytest.approx((50.0 + 2 * P) / (1 - 0.652))
    assert g.iy == pytest.approx(g.ix)
    assert g.a2 - g.a1 == pytest.approx(g.ix) and g.a1 == pytest.approx(-g.a2)


def test_ray_grid_and_areas(orc):
    g = orc.geometry(0.45, 0.05, 0.45, 25.0, 512, rays_per_pixel=100.0)
    # near-square ray cells, ray count within rounding of N_av N_pix
    assert abs(g.ray_dx / g.ray_dy - 1.0) < 2.0 / min(g.nx, g.ny)
    assert abs(g.n_rays / (100.0 * 512 ** 2) - 1.0) < 2.0 / min(g.nx, g.ny)
    assert g.s_img * g.n_rays == pytest.approx(g.ix * g.iy)
    assert g.s_src * g.npix ** 2 == pytest.approx(25.0 ** 2)


def test_level_resolutions(orc):
    frac = GOLDEN["level1_short_side_fraction"]["value"]
    ratio = GOLDEN["level2_ratio"]["value"]
    g0 = orc.geometry(0.3, 0.0, 0.3, 10.0, 256, n_rays=2048 ** 2)
    # few lenses: dx1 limited by the short side
    g = g0.with_lens_count(105)
    assert g.dx1 == pytest.approx(min(g.ix, g.iy) * frac)
    # many lenses: dx1 = L0 = sqrt(I_x I_y / N_*)
    g = g0.with_lens_count(100000)
    assert g.dx1 == pytest.approx(math.sqrt(g.ix * g.iy / 100000))
    assert g.dx2 == pytest.approx(g.dx1 / ratio) and g.q == int(ratio)
    # level-1 cells tile the rectangle and are no larger than dx1
    assert g.ix / g.n1x <= g.dx1 * (1 + 1e-12) and g.iy / g.n1y <= g.dx1 * (1 + 1e-12)
    assert (g.n1x - 1) * g.dx1 < g.ix


def test_critical_line_rejected(orc):
    with pytest.raises(orc.CriticalLineError):
        orc.geometry(0.5, 0.0, 0.5, 100.0, 64, rays_per_pixel=10.0)
    g = orc.geometry(0.5, 0.05, 0.5, 100.0, 64, rays_per_pixel=10.0)
    assert g.mu_th == pytest.approx(1.0 / ((1 - 0.55) ** 2 - 0.25))


def test_lens_count_rule_roundtrip(orc):
    S = orc.source_side_for_lens_count(0.6, 0.0, 0.6, 1_000_000)
    g = orc.geometry(0.6, 0.0, 0.6, S, 10000, rays_per_pixel=1000.0)
    assert abs(g.n_stars_expected - 1_000_000) <= 1
    assert S == pytest.approx(synth.configs.CFG3.source_side, rel=1e-4)


def test_generator_deterministic_and_uniform():
    r1 = synth.uniform01(5, 0, 100000)
    r2 = synth.uniform01(5, 0, 1000, offset=500)
    assert np.array_equal(r1[500:1500], r2)
    assert 0.0 <= r1.min() and r1.max() < 1.0
    assert abs(r1.mean() - 0.5) < 0.005 and abs(r1.var() - 1 / 12) < 0.002
    assert not np.array_equal(synth.uniform01(5, 1, 100), synth.uniform01(5, 0, 100))


def test_salpeter_masses():
    L = synth.uniform_lenses(400000, (-1, 1, -2, 2), 9, mass="salpeter", m_min=0.1, m_max=1.0)
    assert abs(L.m.mean() - 1.0) < 0.01                  # normalised to <M>
    mean = synth.salpeter_mean_mass(0.1, 1.0)
    assert mean == pytest.approx(0.22340, abs=2e-5)      # analytic <M> for [0.1, 1]
    Mabs = L.m * mean
    assert Mabs.min() >= 0.1 - 1e-12 and Mabs.max() <= 1.0 + 1e-12
    # CDF check: fraction below 0.2 M_sun
    a = 1 - 2.35
    frac = (0.2 ** a - 0.1 ** a) / (1.0 ** a - 0.1 ** a)
    assert abs(np.mean(Mabs < 0.2) - frac) < 0.003
    assert L.x.min() >= -1 and L.x.max() < 1 and L.y.min() >= -2 and L.y.max() < 2


def test_batch_draws():
    d = synth.configs.batch_draws()
    assert len(d) == 64
    for b in d:
        k = b.kappa_star + b.kappa_c
        assert min(abs(1 - k - b.gamma), abs(1 - k + b.gamma)) >= 0.05
        assert 1000 <= b.n_star_target <= 100000 and b.npix in (1024, 2048, 4096)
    assert d == synth.configs.batch_draws()
