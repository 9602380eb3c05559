"""The learned interpolant on the GPU: network forward and gradients against
the FP64 oracle, exact corner data and samples against the oracle's far field,
training (loss falls, the network beats the coarse grid without it), rays
against the oracle and the direct sum, and the grid-interpolation fallback."""
import numpy as np
import pytest

import oracle as orc
from oracle import learned as ol
import synth
from gpu_common import THREADS

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def irs():
    import paper_2204_10871_amd as irs
    irs.load()
    return irs


def bf16_round(x):
    """Round float32 values to the nearest BF16 (ties to even), kept as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


def _net(seed=3, scale=0.1, fscale=1.0):
    fr = synth.network.fourier_frequencies(seed, fscale)
    th = bf16_round(synth.network.random_parameters(seed, scale))
    return fr, th


# BF16 has a unit roundoff u = 2^-9.  Each of the five products rounds its
# inputs (features or activations, and weights) to BF16 and accumulates in
# FP32, so an output differs from the FP64 network by at most about
# 5 * 2u = 0.02 of its absolute-value scale sum_k |W_ok| |a_k| + |b_o| (the
# scale of the last product, which bounds the propagated errors as well for
# these O(1) random layers); the tests allow 0.03.
FWD_TOL = 0.03


def test_mlp_forward_matches_oracle(irs):
    import torch
    fr, th = _net()
    n = 1000                                   # not a multiple of 64
    rng = np.random.default_rng(1)
    h = rng.uniform(0, 1, (n, 2))
    hd = torch.tensor(h.T.astype(np.float32).copy(), device="cuda:0")
    yd = torch.empty((16, n), dtype=torch.float32, device="cuda:0")
    irs.mlp_forward(fr, th, hd, yd)
    y = yd.cpu().numpy().T.astype(np.float64)
    yo, cache = ol.forward(th.astype(np.float64), fr.astype(np.float64), h.astype(np.float32))
    P = ol.unpack(th.astype(np.float64))
    scale = np.abs(cache[4]) @ np.abs(P[8]).T + np.abs(P[9])
    err = np.abs(y - yo) / scale
    say(f"forward: max |dy|/scale {err.max():.3e}, mean {err.mean():.3e}")
    assert err.max() < FWD_TOL


def test_learned_weights_match_oracle(irs):
    """The weights the rays take (irs_learn_weights: the BF16 network
    tabulated at the 33 x 33 nodes and blended) against the oracle's FP64
    table blend, at random offsets, the square's edges and offsets a rounding
    step outside it.  The blend is a convex combination of node values, so
    its error is at most the blend of the nodes' FWD_TOL bounds."""
    import torch
    fr, th = _net()
    p, L, og = _plan(irs, npix=32, n_rays=20_000)
    rng = np.random.default_rng(4)
    h = rng.uniform(0, 1, (2000, 2))
    h[:6] = [[0, 0], [1, 1], [1, 0], [0, 1], [-1e-7, 0.5], [0.5, 1 + 1e-7]]
    with irs.Plan(p, L.x, L.y, L.m) as pl:
        pl.learn_set(fr, th, irs.learn_params(coarse=4, n_val=2000, train_rows=2))
        hd = torch.tensor(h.T.astype(np.float32).copy(), device="cuda:0")
        yd = torch.empty((16, h.shape[0]), dtype=torch.float32, device="cuda:0")
        pl.learn_weights(hd, yd)
        y = yd.cpu().numpy().T.astype(np.float64)
    th64, fr64 = th.astype(np.float64), fr.astype(np.float64)
    h32 = h.astype(np.float32).astype(np.float64)
    yo = ol.table_weights(th64, fr64, h32)
    _, cache = ol.forward(th64, fr64, ol.table_nodes())
    P = ol.unpack(th64)
    scale = ol.table_blend(np.abs(cache[4]) @ np.abs(P[8]).T + np.abs(P[9]), h32)
    err = np.abs(y - yo) / scale
    say(f"table weights: max |dy|/scale {err.max():.3e}, mean {err.mean():.3e}")
    assert err.max() < FWD_TOL


def _records(rng, n):
    """Sample records with random h, unit-size D and targets (fields as the
    sample kernel writes them)."""
    f = np.zeros((24, n), np.float32)
    f[0:2] = rng.uniform(0, 1, (2, n))
    D = rng.normal(size=(16, n)) * 0.5
    f[2:18] = D
    f[18:20] = rng.normal(size=(2, n)) * 0.3
    f[20] = 1.0
    return f


@pytest.mark.parametrize("n", [200, 1024])
def test_mlp_gradient_matches_oracle(irs, n):
    """Loss and gradient of the training kernels against the FP64 oracle
    (whose own gradient is pinned by finite differences)."""
    import torch
    fr, th = _net(seed=5)
    rng = np.random.default_rng(n)
    rec = _records(rng, n)
    loss, g = irs.mlp_loss_grad(fr, th, torch.tensor(rec, device="cuda:0"), n)
    h = rec[0:2].T.astype(np.float64)
    D = (rec[2:18:2] + 1j * rec[3:18:2]).T.astype(np.complex128)
    T = (rec[18] + 1j * rec[19]).astype(np.complex128)
    lo, go = ol.loss_and_grad(th.astype(np.float64), fr.astype(np.float64), h, D, T)
    say(f"n={n}: loss {loss:.6e} vs {lo:.6e}")
    assert abs(loss - lo) <= 0.02 * lo
    off = 0
    for k, shp in enumerate(ol._SHAPES):
        m = int(np.prod(shp))
        a, b = g[off:off + m].astype(np.float64), go[off:off + m]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        say(f"  block {k} {shp}: rel {rel:.3e} cos {cos:.6f}")
        assert rel < 0.05 and cos > 0.998
        off += m


# a small map of the learned workload's shape (kappa_* = gamma = 0.5, kappa_c = 0.05)
def _plan(irs, method="learned", S=6.0, npix=64, n_rays=200_000, seed=21, mass="unit"):
    p = irs.make_params(0.5, 0.05, 0.5, S, npix, n_rays=n_rays, method=method, precision="fp64")
    g0 = irs.geometry(p, 0)
    L = synth.uniform_lenses(g0["n_stars_expected"], (g0["a1"], g0["a2"], g0["b1"], g0["b2"]),
                             seed, mass=mass)
    og = orc.geometry(0.5, 0.05, 0.5, S, npix, n_rays=n_rays, n_lens=L.n)
    return p, L, og


@pytest.mark.parametrize("mass", ["unit", "salpeter"])
def test_corners_match_oracle(irs, mass):
    p, L, og = _plan(irs, mass=mass)
    cs, perm = orc.level1(og, L)
    qc = 3
    with irs.Plan(p, L.x, L.y, L.m) as pl:
        g = pl.geometry
        for r0 in (0, g["n1y"] // 2, g["n1y"] - 1):
            A, dA = pl.learn_corners(qc, r0, 1)
            sx = (g["a2"] - g["a1"]) / (g["n1x"] * qc)
            sy = (g["b2"] - g["b1"]) / (g["n1y"] * qc)
            cx = np.repeat(np.arange(g["n1x"]), (qc + 1) ** 2)
            b, a = np.divmod(np.tile(np.arange((qc + 1) ** 2), g["n1x"]), qc + 1)
            x = g["a1"] + (cx * qc + a) * sx
            y = g["b1"] + (r0 * qc + b) * sy
            Ao, dAo = orc.far_point(og, L, cs, perm, cx, np.full_like(cx, r0), x, y, THREADS)
            e1 = np.max(np.abs(A.ravel() - Ao)) / np.max(np.abs(Ao))
            e2 = np.max(np.abs(dA.ravel() - dAo)) / np.max(np.abs(dAo))
            say(f"row {r0}: corner A rel {e1:.2e}, A' rel {e2:.2e}")
            assert e1 < 1e-12 and e2 < 1e-12


def test_samples_match_oracle(irs):
    import torch
    p, L, og = _plan(irs)
    cs, perm = orc.level1(og, L)
    qc, per_cell = 4, 3
    with irs.Plan(p, L.x, L.y, L.m) as pl:
        g = pl.geometry
        r0 = g["n1y"] // 2
        n = g["n1x"] * per_cell
        out = torch.empty((24, n), dtype=torch.float32, device="cuda:0")
        pl.learn_samples(qc, r0, 1, per_cell, 99, out)
        f = out.cpu().numpy().astype(np.float64)
    cx, cy, sq = f[21].astype(np.int64), f[22].astype(np.int64), f[23].astype(np.int64)
    assert np.all(cy == r0) and np.all(np.bincount(cx, minlength=g["n1x"]) == per_cell)
    b, a = np.divmod(sq, qc)
    sx = (g["a2"] - g["a1"]) / (g["n1x"] * qc)
    sy = (g["b2"] - g["b1"]) / (g["n1y"] * qc)
    X0, Y0 = g["a1"] + (cx * qc + a) * sx, g["b1"] + (cy * qc + b) * sy
    h = f[0:2].T
    x, y = X0 + h[:, 0] * sx, Y0 + h[:, 1] * sy
    zc = ol.square_corners(X0, Y0, sx, sy)
    Ac, dAc = orc.far_point(og, L, cs, perm, np.repeat(cx, 4), np.repeat(cy, 4),
                            zc.real.ravel(), zc.imag.ravel(), THREADS)
    Ac, dAc = Ac.reshape(-1, 4), dAc.reshape(-1, 4)
    A, _ = orc.far_point(og, L, cs, perm, cx, cy, x, y, THREADS)
    D, sigma = ol.local_data(zc, Ac, dAc, sx, sy)
    T = (A - ol.base_interp(zc, Ac, dAc, h, x + 1j * y)) / sigma
    Dg = f[2:18:2].T + 1j * f[3:18:2].T
    Tg = f[18] + 1j * f[19]
    eD = np.max(np.abs(Dg - D))
    eT = np.max(np.abs(Tg - T))
    es = np.max(np.abs(f[20] - sigma) / sigma)
    say(f"samples: D {eD:.2e}, T {eT:.2e}, sigma rel {es:.2e}, |T| max {np.abs(T).max():.3f}")
    assert eD < 1e-6 and eT < 1e-5 * max(1.0, np.abs(T).max()) and es < 1e-6


LEARN_SMALL = dict(coarse=12, train_rows=6, n_samples=500_000, n_val=50_000, batch=8192,
                   steps=3000, lr=2e-3, lr_final=2e-5)


@pytest.fixture(scope="module")
def trained(irs):
    """A small learned plan, trained once for the tests below."""
    p, L, og = _plan(irs, S=10.0, npix=96, n_rays=400_000)
    pl = irs.Plan(p, L.x, L.y, L.m)
    fr = synth.network.fourier_frequencies(7)
    rep = pl.learn(fr, irs.learn_params(**LEARN_SMALL))
    say("training report: " + ", ".join(f"{k}={v:.4g}" if isinstance(v, float) else f"{k}={v}"
                                       for k, v in rep.items()))
    yield pl, p, L, og, rep
    pl.close()


def test_training_reduces_loss_and_beats_base(trained):
    """The gain: on the same coarse grid (12 x 12 squares per level-1 cell,
    169 exact corner values against the paper's 400 level-2 points) the grid
    alone misses the tolerance many times over; with the network it meets it."""
    pl, p, L, og, rep = trained
    assert rep["loss_last"] < 0.01 * rep["loss_first"]
    assert rep["val_mean_abs"] < 0.05 * rep["base_mean_abs"]
    assert rep["val_p9999_abs"] < 0.05 * rep["base_p9999_abs"]
    assert rep["base_mean_abs"] > 10 * rep["tol_mean"]
    assert rep["fallback"] == 0


def test_learned_rays_match_oracle_and_direct(irs, trained):
    """Per-ray alpha of the learned path against the oracle's learned rays
    (FP64 network with the trained weights) and against the direct sum."""
    pl, p, L, og, rep = trained
    fr, th, qc = pl.learn_get()
    cs, perm = orc.level1(og, L)
    rng = np.random.default_rng(3)
    ids = np.sort(rng.choice(pl.n_rays, 3000, replace=False))
    a1 = np.empty(ids.size)
    a2 = np.empty(ids.size)
    px = np.empty(ids.size, np.int64)
    for k, r in enumerate(ids):                   # single rays: any index works
        x1, x2, pp = pl.deflect_grid(int(r), 1)
        a1[k], a2[k], px[k] = x1[0], x2[0], pp[0]
    ref = orc.shoot_direct(og, L, ray_ids=ids, threads=THREADS, want_counts=False)
    d = np.hypot(a1 - ref["alpha1"], a2 - ref["alpha2"])
    rel = d / np.hypot(ref["alpha1"], ref["alpha2"])
    mis = int(np.sum(px != ref["pix"]))
    say(f"learned vs direct: max |d alpha| {d.max():.2e}, mean {d.mean():.2e}, "
        f"max rel {rel.max():.2e}, pixel mismatches {mis}/{ids.size}, fallback {rep['fallback']}")
    if rep["fallback"]:
        pytest.skip("the network missed the tolerance; the fallback is tested separately")
    assert rel.max() < 1e-4
    assert mis <= 1
    oa1, oa2, opx = ol.learned_rays(og, L, cs, perm, qc, fr.astype(np.float64),
                                    th.astype(np.float64), ids, THREADS)
    do = np.hypot(a1 - oa1, a2 - oa2)
    say(f"learned vs oracle-learned: max |d alpha| {do.max():.2e}")
    # the two differ by the BF16 network's error, a fraction FWD_TOL of the
    # correction it computes; the correction is at most the base error
    assert do.max() <= FWD_TOL * rep["base_max_abs"] + 1e-12


def test_learned_rays_independent_of_the_call(irs, trained):
    """A lane of the learned ray kernel takes four rows of one column, and
    nothing is shared between rows but loads, so a ray's alpha and pixel are
    the same bits whether it is shot alone or inside whole rows: here every
    ray of rows that straddle level-1 cell rows, against single-ray calls."""
    pl, p, L, og, rep = trained
    if rep["fallback"]:
        pytest.skip("the network missed the tolerance; the fallback is tested separately")
    g = pl.geometry
    nx = g["nx"]
    j0, _ = pl.level1_row_rays(g["n1y"] // 2)       # a level-1 row's first ray row
    first = (j0 - 3) * nx                           # rows j0-3 .. j0+2: two cell rows
    n = 6 * nx
    a1, a2, px = pl.deflect_grid(first, n)
    rng = np.random.default_rng(8)
    ids = np.sort(rng.choice(n, 600, replace=False))
    for k in ids:
        b1, b2, bp = pl.deflect_grid(first + int(k), 1)
        assert (a1[k], a2[k], px[k]) == (b1[0], b2[0], bp[0]), int(k)
    say(f"learned rows {j0 - 3}..{j0 + 2}: {n} rays, 600 single-ray calls identical")


def test_learned_map_vs_direct(irs, trained):
    """Whole map: the learned map against the direct-sum map (the reference)."""
    pl, p, L, og, rep = trained
    if rep["fallback"]:
        pytest.skip("the network missed the tolerance; the fallback is tested separately")
    counts, st = pl.shoot_map()
    assert st["learned"] == 1
    pd = irs.make_params(0.5, 0.05, 0.5, 10.0, 96, n_rays=400_000, method="direct",
                         precision="fp64")
    with irs.Plan(pd, L.x, L.y, L.m) as dp:
        ref, _ = dp.shoot_map()
    c, r = counts.astype(np.int64), ref.astype(np.int64)
    l1 = np.abs(c - r).sum() / r.sum()
    say(f"learned map vs direct: rel-L1 {l1:.3e}, rays landed {c.sum()} vs {r.sum()}")
    assert l1 <= 1e-3
    again, _ = pl.shoot_map()
    assert np.array_equal(again, counts)


def test_fallback_is_the_grid_interpolation(irs):
    """An unreachable tolerance engages the fallback: the map is the grid
    interpolation's, bit for bit."""
    p, L, og = _plan(irs)
    fr = synth.network.fourier_frequencies(7, 1.0)
    lp = irs.learn_params(coarse=2, train_rows=2, n_samples=4096, n_val=2048, batch=1024,
                          steps=10, tol_mean=1e-30)
    with irs.Plan(p, L.x, L.y, L.m) as pl:
        rep = pl.learn(fr, lp)
        assert rep["fallback"] == 1
        counts, st = pl.shoot_map()
        assert st["learned"] == 0
    pi = irs.make_params(0.5, 0.05, 0.5, 6.0, 64, n_rays=200_000, method="interp",
                         precision="fp64")
    with irs.Plan(pi, L.x, L.y, L.m) as ip:
        ref, _ = ip.shoot_map()
    assert np.array_equal(counts, ref)


def test_untrained_learned_plan_is_an_error(irs):
    p, L, og = _plan(irs)
    with irs.Plan(p, L.x, L.y, L.m) as pl:
        with pytest.raises(irs.IrsError) as e:
            pl.shoot_map()
        assert e.value.status == 1


def test_learn_set_roundtrip(irs, trained):
    """A saved network installed on a fresh plan gives the same map."""
    pl, p, L, og, rep = trained
    fr, th, qc = pl.learn_get()
    counts, _ = pl.shoot_map()
    with irs.Plan(p, L.x, L.y, L.m) as p2:
        rep2 = p2.learn_set(fr, th, irs.learn_params(**dict(LEARN_SMALL, coarse=qc)))
        assert rep2["fallback"] == rep["fallback"]
        c2, _ = p2.shoot_map()
    assert np.array_equal(c2, counts)
