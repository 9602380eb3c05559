"""Pins of the learned interpolant's FP64 reference (oracle/learned.py) and of
the exact far field at arbitrary points (orc_far_point)."""
import math

import numpy as np
import pytest

import oracle as orc
from oracle import learned as ol
import synth


def _random_theta(rng, scale=0.2):
    return rng.normal(0.0, scale, ol.N_PARAMS)


def test_param_count():
    assert ol.N_PARAMS == 4 * (128 * 128 + 128) - 128 * 128 + 128 * 128 + 16 * 128 + 16
    assert ol.N_PARAMS == 68112


def test_backward_matches_finite_differences():
    """Central differences of the FP64 loss pin the reverse-mode gradient."""
    rng = np.random.default_rng(1)
    theta = _random_theta(rng)
    freqs = rng.normal(0.0, 1.0, (64, 2))
    n = 7
    h = rng.uniform(0, 1, (n, 2))
    D = rng.normal(size=(n, 8)) + 1j * rng.normal(size=(n, 8))
    T = rng.normal(size=n) + 1j * rng.normal(size=n)
    loss, g = ol.loss_and_grad(theta, freqs, h, D, T)
    # coordinates from every block: weights and biases of all five layers
    offs, o = [], 0
    for s in ol._SHAPES:
        k = int(np.prod(s))
        offs += list(o + rng.choice(k, 6, replace=False))
        o += k
    eps = 1e-6
    for i in offs:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (ol.loss_and_grad(tp, freqs, h, D, T)[0] - ol.loss_and_grad(tm, freqs, h, D, T)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_special_cases():
    """Zero weights give y = b5; identity hidden layers give y = W5 relu(phi) + b5,
    with phi written out with scalar sin/cos."""
    rng = np.random.default_rng(2)
    freqs = rng.normal(0.0, 1.5, (64, 2))
    h = rng.uniform(0, 1, (5, 2))
    theta = np.zeros(ol.N_PARAMS)
    P = ol.unpack(theta)
    P[-1][:] = np.arange(16) * 0.25 - 1.0
    y, _ = ol.forward(theta, freqs, h)
    assert np.array_equal(y, np.tile(P[-1], (5, 1)))

    theta = np.zeros(ol.N_PARAMS)
    P = ol.unpack(theta)
    for l in range(4):
        P[2 * l][:] = np.eye(128)
    P[8][:] = rng.normal(size=(16, 128))
    P[9][:] = rng.normal(size=16)
    y, _ = ol.forward(theta, freqs, h)
    for s in range(5):
        phi = []
        for j in range(64):
            t = 2 * math.pi * (freqs[j, 0] * (h[s, 0] - 0.5) + freqs[j, 1] * (h[s, 1] - 0.5))
            phi.append(math.sin(t))
        for j in range(64):
            t = 2 * math.pi * (freqs[j, 0] * (h[s, 0] - 0.5) + freqs[j, 1] * (h[s, 1] - 0.5))
            phi.append(math.cos(t))
        for o in range(16):
            ref = P[9][o] + sum(P[8][o, k] * max(phi[k], 0.0) for k in range(128))
            assert abs(y[s, o] - ref) < 1e-12


def _square(rng, n):
    x0 = rng.uniform(-5, 5, n)
    y0 = rng.uniform(-5, 5, n)
    sx, sy = 0.3, 0.2
    return ol.square_corners(x0, y0, sx, sy), sx, sy


def test_base_interpolant_linear_and_quadratic():
    """Exact on linear fields; on A = a (z - z_m)^2 its error is
    sum_c w_c u_c^2 - u^2 (u = z - z_m), which is (sx^2 - sy^2)/4 at the centre
    and zero at the corners."""
    rng = np.random.default_rng(3)
    zc, sx, sy = _square(rng, 40)
    h = rng.uniform(0, 1, (40, 2))
    z = zc[:, 0] + h[:, 0] * sx + 1j * h[:, 1] * sy
    a, b = 1.3 - 0.4j, -0.7 + 2.1j
    I = ol.base_interp(zc, a + b * zc, np.full_like(zc, b), h, z)
    assert np.max(np.abs(I - (a + b * z))) < 1e-12
    c2 = 0.8 + 0.3j
    zm = zc.mean(axis=1)
    A = lambda zz, m: c2 * (zz - m) ** 2
    I = ol.base_interp(zc, A(zc, zm[:, None]), 2 * c2 * (zc - zm[:, None]), h, z)
    u, uc = z - zm, zc - zm[:, None]
    err = c2 * (np.sum(ol.bilinear(h) * uc ** 2, axis=1) - u ** 2)
    assert np.max(np.abs((A(z, zm) - I) - err)) < 1e-12
    hc = np.full((40, 2), 0.5)
    Ic = ol.base_interp(zc, A(zc, zm[:, None]), 2 * c2 * (zc - zm[:, None]), hc, zm)
    assert np.max(np.abs((A(zm, zm) - Ic) - c2 * (sx ** 2 - sy ** 2) / 4)) < 1e-12
    for c, hh in enumerate([(0, 0), (1, 0), (0, 1), (1, 1)]):
        hk = np.tile(np.array(hh, float), (40, 1))
        Ik = ol.base_interp(zc, A(zc, zm[:, None]), 2 * c2 * (zc - zm[:, None]), hk, zc[:, c])
        assert np.max(np.abs(Ik - A(zc[:, c], zm))) < 1e-12


def test_table_nodes_and_blend():
    """The rays' weight table: node b (T+1) + a sits at (a/T, b/T); the blend
    returns a node's values at the node, reproduces any bilinear function
    c0 + c1 hx + c2 hy + c3 hx hy exactly (different coefficients per output,
    so a swapped axis or a shifted node fails), clamps offsets outside the
    square, and on a smooth function stays within the bilinear bound
    (d^2/8)(max|f_xx| + max|f_yy|), d = 1/T."""
    T = ol.TABLE_SIDE
    nodes = ol.table_nodes()
    assert nodes.shape == ((T + 1) ** 2, 2)
    a, b = 5, 17
    assert np.array_equal(nodes[b * (T + 1) + a], [a / T, b / T])
    rng = np.random.default_rng(11)
    c = rng.normal(size=(4, 16))
    f = lambda h: (c[0] + np.outer(h[:, 0], c[1]) + np.outer(h[:, 1], c[2])
                   + np.outer(h[:, 0] * h[:, 1], c[3]))
    Y = f(nodes)
    assert np.array_equal(ol.table_blend(Y, nodes), Y)
    h = rng.uniform(0, 1, (500, 2))
    h[:4] = [[0, 0], [1, 1], [1, 0], [0.5, 1]]               # edges of the square
    assert np.max(np.abs(ol.table_blend(Y, h) - f(h))) < 1e-13
    out = np.array([[-0.25, 0.3], [1.5, 0.3], [0.7, -1e-9], [0.7, 1 + 1e-9]])
    assert np.allclose(ol.table_blend(Y, out), f(np.clip(out, 0, 1)), rtol=0, atol=1e-13)
    k1, k2 = 2 * np.pi * 1.3, 2 * np.pi * 0.7
    g = lambda h: np.sin(k1 * h[:, 0] + k2 * h[:, 1])[:, None]
    err = np.abs(ol.table_blend(g(nodes), h) - g(h)).max()
    bound = (1.0 / T) ** 2 / 8 * (k1 ** 2 + k2 ** 2)
    assert 0.05 * bound < err <= bound


def test_learned_value_uses_the_table():
    """learned_value's correction is sigma sum_k L_k D_k with L the blended
    table of the network's outputs: at a node it equals the network's own."""
    rng = np.random.default_rng(12)
    th = _random_theta(rng)
    fr = rng.normal(0, 0.25, (64, 2))
    zc, sx, sy = _square(rng, 6)
    Ac = rng.normal(size=(6, 4)) + 1j * rng.normal(size=(6, 4))
    dAc = rng.normal(size=(6, 4)) + 1j * rng.normal(size=(6, 4))
    T = ol.TABLE_SIDE
    h = np.array([[3, 7], [0, 0], [T, T], [12, 31], [31, 1], [16, 16]], float) / T
    z = zc[:, 0] + h[:, 0] * sx + 1j * h[:, 1] * sy
    D, sigma = ol.local_data(zc, Ac, dAc, sx, sy)
    want = ol.base_interp(zc, Ac, dAc, h, z) + sigma * ol.predict(th, fr, h, D)
    got = ol.learned_value(th, fr, zc, Ac, dAc, sx, sy, h, z)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))


def test_local_data_invariants():
    """delta and eps sum to zero over the corners, vanish for linear fields
    (up to rounding), and a quadratic field's delta equals 2 a u_c s."""
    rng = np.random.default_rng(4)
    zc, sx, sy = _square(rng, 30)
    c2 = 0.5 - 1.1j
    zm = zc.mean(axis=1, keepdims=True)
    Ac = c2 * (zc - zm) ** 2 + 3.0
    dAc = 2 * c2 * (zc - zm)
    D, sigma = ol.local_data(zc, Ac, dAc, sx, sy)
    assert np.max(np.abs(D[:, :4].sum(axis=1))) < 1e-12
    assert np.max(np.abs(D[:, 4:].sum(axis=1))) < 1e-12
    s = 0.5 * (sx + sy)
    assert np.max(np.abs(D[:, :4] * sigma[:, None] - 2 * c2 * (zc - zm) * s)) < 1e-12
    assert np.all(np.max(np.abs(D), axis=1) <= 1 + 1e-12)


@pytest.fixture(scope="module")
def far_case():
    g = orc.geometry(0.45, 0.05, 0.45, 6.0, 32, n_rays=20000)
    rect = (g.a1, g.a2, g.b1, g.b2)
    L = synth.uniform_lenses(g.n_stars_expected, rect, 77)
    cs, perm = orc.level1(g, L)
    return g, L, cs, perm


def _points(g, rng, n, corner=False):
    w1 = (g.a2 - g.a1) / g.n1x
    h1 = (g.b2 - g.b1) / g.n1y
    if corner:
        cx = rng.choice([0, g.n1x - 1], n)
        cy = rng.choice([0, g.n1y - 1], n)
    else:
        cx = rng.integers(1, g.n1x - 1, n)
        cy = rng.integers(1, g.n1y - 1, n)
    x = g.a1 + (cx + rng.uniform(0, 1, n)) * w1
    y = g.b1 + (cy + rng.uniform(0, 1, n)) * h1
    return cx, cy, x, y


def _near(g, L, cs, perm, cx, cy, x, y):
    m = L.masses()
    out = np.zeros(x.size, complex)
    for k in range(x.size):
        for ry in range(cy[k] - 1, cy[k] + 2):
            for rx in range(cx[k] - 1, cx[k] + 2):
                if 0 <= rx < g.n1x and 0 <= ry < g.n1y:
                    c = ry * g.n1x + rx
                    idx = perm[cs[c]:cs[c + 1]]
                    d = (x[k] - L.x[idx]) + 1j * (y[k] - L.y[idx])
                    out[k] += np.sum(m[idx] * d / np.abs(d) ** 2)
    return out


@pytest.mark.parametrize("corner", [False, True])
def test_far_point_against_direct_definition(far_case, corner):
    """conj(alpha - macro - near) from O-1 equals A - kappa_* conj(z) (A - kappa_* F
    in the corner cells, where A carries no sheet)."""
    g, L, cs, perm = far_case
    rng = np.random.default_rng(5 + corner)
    cx, cy, x, y = _points(g, rng, 40, corner)
    A, _ = orc.far_point(g, L, cs, perm, cx, cy, x, y)
    a1, a2, _ = orc.alpha_points(g, L, x, y)
    near = _near(g, L, cs, perm, cx, cy, x, y)
    rest = (a1 - (g.kappa + g.gamma) * x - near.real) - 1j * (a2 - (g.kappa - g.gamma) * y - near.imag)
    z = x + 1j * y
    if corner:
        I1, I2 = orc.sheet_I((g.a1, g.a2, g.b1, g.b2), x, y)
        ref = A - g.kappa_star * (I1 - 1j * I2) / np.pi
    else:
        ref = A - g.kappa_star * np.conj(z)
    assert np.max(np.abs(rest - ref)) < 1e-11 * max(1.0, np.max(np.abs(rest)))


def test_far_point_derivative_and_analyticity(far_case):
    """A' from central differences along x, and i A' along y (Cauchy-Riemann)."""
    g, L, cs, perm = far_case
    rng = np.random.default_rng(9)
    cx, cy, x, y = _points(g, rng, 30)
    A, dA = orc.far_point(g, L, cs, perm, cx, cy, x, y)
    e = 1e-5
    Ax = (orc.far_point(g, L, cs, perm, cx, cy, x + e, y)[0]
          - orc.far_point(g, L, cs, perm, cx, cy, x - e, y)[0]) / (2 * e)
    Ay = (orc.far_point(g, L, cs, perm, cx, cy, x, y + e)[0]
          - orc.far_point(g, L, cs, perm, cx, cy, x, y - e)[0]) / (2 * e)
    scale = np.max(np.abs(dA))
    assert np.max(np.abs(Ax - dA)) < 1e-7 * scale
    assert np.max(np.abs(Ay - 1j * dA)) < 1e-7 * scale


def test_far_point_continuous_on_the_edges(far_case):
    """Corner points of the top and bottom cell rows lie on the rectangle's
    edges (or a rounding step outside).  The field there must continue the
    interior values: the principal Log's cut runs along those edges, so it
    is taken pointing away from the rectangle instead."""
    g, L, cs, perm = far_case
    cx = np.arange(1, g.n1x - 1)
    x = g.a1 + (cx + 0.37) * (g.a2 - g.a1) / g.n1x
    for cy, yb, sgn in ((g.n1y - 1, g.b2, -1.0), (0, g.b1, 1.0)):
        cyv = np.full_like(cx, cy)
        A_e, dA_e = orc.far_point(g, L, cs, perm, cx, cyv, x, np.full(x.size, yb))
        A_o, dA_o = orc.far_point(g, L, cs, perm, cx, cyv, x, np.full(x.size, yb - sgn * 1e-12))
        A_i, dA_i = orc.far_point(g, L, cs, perm, cx, cyv, x, np.full(x.size, yb + sgn * 1e-7))
        scale = np.max(np.abs(dA_i))
        assert np.max(np.abs(dA_e - dA_i)) < 1e-5 * scale
        assert np.max(np.abs(dA_o - dA_i)) < 1e-5 * scale
        assert np.max(np.abs(A_e - A_i)) < 1e-5 * max(1.0, np.max(np.abs(A_i)))
