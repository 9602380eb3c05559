"""The circular lens plane (Sec. 2.1-2.2, Eq. 9) in the oracle, pinned by
physics the code does not contain: the stars of a uniform disc pull, on
average, like the enclosed mass (Gauss's law: kappa_* theta inside), so the
circle's sheet must cancel them there; and the lens count of the circle
against the rectangle."""
import math

import numpy as np

import oracle
import synth


def test_disc_sheet_cancels_the_mean_star_field():
    # average over lens draws of alpha - (kappa + gamma, kappa - gamma) theta
    # (the stars plus the sheet) at interior points: zero if the sheet is
    # -kappa_* theta; a sign slip would leave 2 kappa_* theta, a missing
    # sheet kappa_* theta (both ~3 at |theta| = 10)
    g = oracle.geometry(0.3, 0.0, 0.3, 10.0, 64, n_rays=64 * 64, circle=True)
    R, n = g.lens_radius, g.n_stars_expected
    pts = np.array([[10.0, 0.0], [0.0, 8.0], [-7.0, 6.0], [18.0, -9.0], [-20.0, -5.0]])
    acc = np.zeros_like(pts)
    draws = 400
    for s in range(draws):
        L = synth.disc_lenses(n, R, 5000 + s)
        a1, a2, _ = oracle.alpha_points(g, L, pts[:, 0], pts[:, 1])
        acc[:, 0] += a1 - (g.kappa + g.gamma) * pts[:, 0]
        acc[:, 1] += a2 - (g.kappa - g.gamma) * pts[:, 1]
    mean = acc / draws
    # the perturbation's spread is a few phi_0 = sqrt(kappa_*) per draw
    assert np.all(np.abs(mean) < 0.35), mean
    # and the stars alone do pull with kappa_* theta on average
    g0 = oracle.geometry(0.3, 0.0, 0.3, 10.0, 64, n_rays=64 * 64, circle=True, sheet=False)
    acc0 = np.zeros_like(pts)
    for s in range(draws):
        L = synth.disc_lenses(n, R, 5000 + s)
        a1, a2, _ = oracle.alpha_points(g0, L, pts[:, 0], pts[:, 1])
        acc0[:, 0] += a1 - (g0.kappa + g0.gamma) * pts[:, 0]
        acc0[:, 1] += a2 - (g0.kappa - g0.gamma) * pts[:, 1]
    assert np.all(np.abs(acc0 / draws - 0.3 * pts) < 0.35)


def test_circle_lens_count_is_the_circumscribed_disc():
    # the circle circumscribes the image rectangle; at density kappa_*/pi it
    # holds kappa_* R^2 lenses against kappa_* I_x I_y / pi for the rectangle
    for ks, kc, gm, S in ((0.3, 0.0, 0.3, 10.0), (0.45, 0.05, 0.45, 25.0)):
        gr = oracle.geometry(ks, kc, gm, S, 64, n_rays=4096)
        gc = oracle.geometry(ks, kc, gm, S, 64, n_rays=4096, circle=True)
        assert math.isclose(gc.lens_radius ** 2, (gr.ix ** 2 + gr.iy ** 2) / 4, rel_tol=1e-14)
        ratio = gc.n_stars_expected / gr.n_stars_expected
        aspect = gr.ix / gr.iy
        assert math.isclose(ratio, math.pi * (aspect + 1 / aspect) / 4, rel_tol=2e-3)
