"""The C-ABI library without a GPU: it loads, exports every function that
include/irs.h declares, derives the same geometry as the oracle, and rejects
bad arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "irs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(irs_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def irs():
    import paper_2204_10871_amd as irs
    irs.load()
    return irs


def test_exports_every_declared_symbol(irs):
    lib = C.CDLL(os.path.join(ROOT, "paper_2204_10871_amd", "libirs.so"))
    names = _declared()
    assert set(names) == set(irs.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


CASES = [
    dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=256, n_rays=2048 ** 2),
    dict(kappa_star=0.45, kappa_c=0.05, gamma=0.45, source_side=25.0, npix=4096,
         rays_per_pixel=100.0, level2_ray_multiple=16.0),
    dict(kappa_star=0.6, kappa_c=0.0, gamma=0.6, source_side=1007.8, npix=10000,
         rays_per_pixel=1000.0),
    dict(kappa_star=0.0, kappa_c=0.23, gamma=0.11, source_side=3.7, npix=37, n_rays=611 * 577,
         border=0.37),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("n_lens", [0, 105, 100000])
def test_geometry_matches_oracle(irs, orc, case, n_lens):
    p = irs.make_params(**case)
    g = irs.geometry(p, n_lens)
    o = orc.geometry(case["kappa_star"], case["kappa_c"], case["gamma"], case["source_side"],
                     case["npix"], rays_per_pixel=case.get("rays_per_pixel"),
                     n_rays=case.get("n_rays"), border=case.get("border"), n_lens=n_lens,
                     level2_ray_multiple=case.get("level2_ray_multiple"))
    for k in ("ix", "iy", "a1", "a2", "b1", "b2", "dx3", "dx1", "dx2", "dpix", "s_img",
              "s_src", "mu_th", "border"):
        assert g[k] == pytest.approx(getattr(o, k), rel=1e-14, abs=1e-300), k
    for k in ("nx", "ny", "n1x", "n1y", "q"):
        assert g[k] == getattr(o, k), k
    assert g["n_stars_expected"] == o.n_stars_expected
    assert g["ray_dx"] == o.ray_dx and g["ray_dy"] == o.ray_dy


@pytest.mark.parametrize("case", CASES[:2])
def test_circle_geometry_matches_oracle(irs, orc, case):
    g = irs.geometry(irs.make_params(circle=True, **case), 0)
    o = orc.geometry(case["kappa_star"], case["kappa_c"], case["gamma"], case["source_side"],
                     case["npix"], rays_per_pixel=case.get("rays_per_pixel"),
                     n_rays=case.get("n_rays"), border=case.get("border"),
                     level2_ray_multiple=case.get("level2_ray_multiple"), circle=True)
    assert g["lens_radius"] == pytest.approx(o.lens_radius, rel=1e-14)
    assert g["n_stars_expected"] == o.n_stars_expected
    assert irs.geometry(irs.make_params(**case), 0)["lens_radius"] == 0.0


def test_circle_needs_the_fp64_direct_sum(irs):
    kw = dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=64,
              rays_per_pixel=10.0, circle=True)
    irs.geometry(irs.make_params(**kw))
    for over in (dict(method="interp"), dict(method="learned"), dict(precision="fp32")):
        with pytest.raises(irs.IrsError) as e:
            irs.geometry(irs.make_params(**{**kw, **over}))
        assert e.value.status == 5                  # IRS_E_UNSUPPORTED


def test_argument_errors(irs):
    with pytest.raises(irs.IrsError) as e:
        irs.geometry(irs.make_params(0.5, 0.0, 0.5, 100.0, 64, rays_per_pixel=10.0))
    assert e.value.status == 2                      # IRS_E_CRITICAL
    for bad in (dict(npix=0), dict(source_side=-1.0), dict(kappa_star=float("nan")),
                dict(rays_per_pixel=0.0)):
        kw = dict(kappa_star=0.3, kappa_c=0.0, gamma=0.3, source_side=10.0, npix=64,
                  rays_per_pixel=10.0)
        kw.update(bad)
        with pytest.raises(irs.IrsError) as e:
            irs.geometry(irs.make_params(**kw))
        assert e.value.status == 1                  # IRS_E_INVALID
    with pytest.raises(irs.IrsError) as e:
        irs.geometry(irs.make_params(0.3, 0.0, 0.3, 10.0, 64, rays_per_pixel=10.0, method=7))
    assert e.value.status == 5                      # IRS_E_UNSUPPORTED


def test_plan_rejects_bad_lenses_before_device(irs):
    """Validation happens on the host: NaN positions fail with IRS_E_INVALID
    and no handle is returned (no device call is made)."""
    p = irs.make_params(0.3, 0.0, 0.3, 10.0, 64, rays_per_pixel=10.0)
    with pytest.raises(irs.IrsError) as e:
        irs.Plan(p, np.array([0.0, np.nan]), np.array([0.0, 1.0]))
    assert e.value.status == 1
    with pytest.raises(irs.IrsError) as e:
        irs.Plan(p, np.array([0.0]), np.array([0.0]), m=np.array([-1.0]))
    assert e.value.status == 1


@pytest.mark.parametrize("method", ["interp", "learned"])
def test_interpolated_plans_reject_lenses_off_the_rectangle(irs, method):
    """The distant-field series assume every lens inside its level-1 cell: a
    lens outside the rectangle fails on the host (no device call is made)."""
    p = irs.make_params(0.3, 0.0, 0.3, 10.0, 64, rays_per_pixel=10.0, method=method)
    g = irs.geometry(p, 2)
    for x, y in ((g["a2"] + 0.01 * g["ix"], 0.0), (0.0, g["b1"] - 1e3), (1e60, 0.0)):
        with pytest.raises(irs.IrsError) as e:
            irs.Plan(p, np.array([0.0, x]), np.array([0.0, y]))
        assert e.value.status == 1
        assert "inside the lens rectangle" in str(e.value)


def test_learned_entry_points_reject_bad_arguments(irs):
    """Argument checks of the learned interpolant's entry points (no device work)."""
    import ctypes as C
    from paper_2204_10871_amd import _ffi
    lib = irs.load()
    lp = irs.learn_params()
    assert 1 <= lp.coarse <= 32 and lp.batch % 256 == 0 and lp.steps > 0
    rep = _ffi.LearnReport()
    assert lib.irs_learn(None, C.byref(lp), None, None, C.byref(rep)) == 1
    assert lib.irs_learn_set(None, None, None, None, None) == 1
    assert lib.irs_learn_get(None, None, None, None) == 1
    assert lib.irs_learn_corners(None, 3, 0, 1, None) == 1
    assert lib.irs_learn_samples(None, 3, 0, 1, 1, 0, None) == 1
    assert lib.irs_mlp_forward(-1, None, None, None, None, None) == 1
    assert lib.irs_mlp_loss_grad(0, None, None, None, None, None, None) == 1
