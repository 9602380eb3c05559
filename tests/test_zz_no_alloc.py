"""irs_shoot_rows_noalloc (the entry point for callers that cannot allocate)
against irs_shoot_rows: the same counts bit for bit, on two calls in a row
with the second on fewer rows, for direct and interpolated plans; and its
refusals, which launch nothing."""
import numpy as np
import pytest

from gpu_common import Case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def irs():
    import paper_2204_10871_amd as irs
    irs.load()
    return irs


def say(msg):
    print(msg, flush=True)


def _compare(pl, npix, row0, nrows):
    import torch
    want = torch.zeros(npix * npix, dtype=torch.int32, device="cuda:0")
    got = torch.full((npix * npix,), 3, dtype=torch.int32, device="cuda:0")
    st = pl.shoot_rows(row0, nrows, want)
    landed = pl.shoot_rows_noalloc(row0, nrows, got)
    torch.cuda.synchronize()
    got -= 3                                   # the call adds, as irs_shoot_rows does
    assert torch.equal(got, want), f"rows {row0}+{nrows}: counts differ"
    assert landed == st["rays_landed"] == int(want.sum().item())
    return landed


CASES = {
    "direct_fp64": dict(args=(0.3, 0.0, 0.3, 6.0, 96), kw=dict(n_rays=700_001, seed=61),
                        method=("direct", "fp64")),
    "direct_fp32": dict(args=(0.45, 0.05, 0.45, 5.0, 128), kw=dict(n_rays=1_000_003, seed=62),
                        method=("direct", "fp32")),
    "interp_fp64": dict(args=(0.35, 0.1, 0.25, 20.0, 96), kw=dict(n_rays=500_000, seed=63),
                        method=("interp", "fp64")),
    "interp_salpeter": dict(args=(0.6, 0.0, 0.6, 12.0, 96),
                            kw=dict(n_rays=900_000, mass="salpeter", seed=64),
                            method=("interp", "fp64")),
}


@pytest.mark.parametrize("name", list(CASES))
def test_noalloc_equals_shoot_rows(irs, name):
    c = CASES[name]
    case = Case(*c["args"], **c["kw"])
    npix = c["args"][4]
    with case.plan(*c["method"]) as pl:
        ny = pl.geometry["ny"]
        say(f"{name}: {pl.geometry['nx']}x{ny} rays, N*={case.lenses.n}")
        if c["method"][0] == "interp":
            pl.shoot_map()                     # sizes the plan's own tables
        first = _compare(pl, npix, 0, ny)      # the whole map
        second = _compare(pl, npix, ny // 3 + 5, ny // 4)   # then fewer rows
        say(f"  landed {first} (whole), {second} (rows {ny // 3 + 5}+{ny // 4})")
        assert second < first


def test_noalloc_refusals(irs):
    import torch
    # an interpolated plan whose tables were never sized: refused, nothing launched
    case = Case(0.35, 0.1, 0.25, 20.0, 96, n_rays=500_000, seed=65)
    counts = torch.zeros(96 * 96, dtype=torch.int32, device="cuda:0")
    with case.plan("interp", "fp64") as pl:
        with pytest.raises(irs.IrsError) as e:
            pl.shoot_rows_noalloc(0, 10, counts)
        assert e.value.status == 1 and "irs_shoot_map" in str(e.value)
    # a level-1 row whose level-2 band does not fit in the static scratch
    big = Case(0.35, 0.1, 0.25, 20.0, 96, n_rays=500_000, seed=66)
    p = irs.make_params(**big.kw, n_rays=500_000, method="interp", precision="fp64",
                        level2_spacing=big.geo.dx1 / 200.0)
    with irs.Plan(p, big.lenses.x, big.lenses.y, big.lenses.m) as pl:
        assert pl.geometry["q"] == 200
        with pytest.raises(irs.IrsError) as e:
            pl.shoot_rows_noalloc(0, 10, counts)
        assert e.value.status == 1 and "scratch" in str(e.value)
    # the learned method is not provided
    with case.plan("learned", "fp64") as pl:
        with pytest.raises(irs.IrsError) as e:
            pl.shoot_rows_noalloc(0, 10, counts)
        assert e.value.status == 5
    torch.cuda.synchronize()
    assert int(counts.sum().item()) == 0
