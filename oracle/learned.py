"""FP64 reference of the learned far-field interpolant.  TEST INFRASTRUCTURE ONLY.

The paper has no learned part: its interpolation (Sec. 2.4) evaluates, for
every ray, a fourth-order Taylor series of the distant-lens field about the
nearest level-2 point.  The learned form keeps the paper's split (near lenses
exact, distant lenses smooth) and replaces that interpolation formula, on a
coarser grid, by a small network.  Inside one level-1 cell the distant-lens
field (plus the analytic part of the sheet) is an analytic function A(z); the
cell is cut into qc x qc squares whose four corners carry A and A'.

For a point z in a square with corners z_c (c = 0: lower left, 1: lower right,
2: upper left, 3: upper right), side lengths (sx, sy), in-square offset
h = ((x - x_0)/sx, (y - y_0)/sy) in [0, 1]^2:

  base interpolant   I(z) = sum_c w_c(h) (A_c + A'_c (z - z_c)),
                     w = ((1-hx)(1-hy), hx(1-hy), (1-hx)hy, hx hy)   (bilinear)
  local data         z_m, A_m, A'_m = means over the corners, s = (sx + sy)/2,
                     delta_c = (A'_c - A'_m) s,
                     eps_c   = A_c - A_m - A'_m (z_c - z_m),
                     sigma   = max_c max(|delta_c|, |eps_c|),
                     D = (delta_0..3, eps_0..3) / sigma     (8 complex numbers)
  network            L(h) in C^8, from the Fourier features of h (below)
  learned value      A(z) ~= I(z) + sigma sum_k L_k(h) D_k.

The correction is linear in the local data (for an analytic field the error of
I is a linear functional of A that vanishes on linear functions), so the network
only has to learn interpolation weights as functions of the position h.

Rays take those weights from a table: L depends on h alone, so the network is
evaluated at the (T+1)^2 nodes (a/T, b/T), a, b = 0..T, T = 32, of the unit
square, and a ray's weights are the bilinear blend of the four nodes around
its h (h clamped to [0, 1]^2; cell (a, b) = (min(floor(T hx), T-1), ...)).
The training fits the network itself; the validation and the rays use the
blended table.

Network (all real):
  phi_j(h)   = sin(2 pi f_j . (h - 1/2)),  phi_{64+j} = cos(2 pi f_j . (h - 1/2)),
               j = 0..63, frequencies f (64 x 2) given;
  a_0 = phi, z_l = W_l a_{l-1} + b_l, a_l = max(z_l, 0) for l = 1..4 (128 wide),
  y = W_5 a_4 + b_5 (16 outputs), L_k = y_{2k} + i y_{2k+1}.
Flat parameter vector: W1 (128 x 128, row = output unit), b1, W2, b2, W3, b3,
W4, b4, W5 (16 x 128), b5 -- 68112 numbers.
Training loss over n samples: (1/n) sum |sum_k L_k D_k - T|^2 with
T = (A(z) - I(z)) / sigma.

Pinned by: central finite differences of the loss (the backward pass), a
closed-form forward special case, the base interpolant's closed-form error
on quadratic fields, and the table blend's exactness on bilinear functions and
its error bound on smooth ones (tests/test_oracle_learned.py).
"""
import numpy as np

N_FREQ = 64
HIDDEN = 128
N_LAYERS = 4
N_OUT = 16
N_DATA = 8

_SHAPES = [(HIDDEN, 2 * N_FREQ), (HIDDEN,)] + [(HIDDEN, HIDDEN), (HIDDEN,)] * (N_LAYERS - 1) \
    + [(N_OUT, HIDDEN), (N_OUT,)]
N_PARAMS = int(sum(np.prod(s) for s in _SHAPES))


def unpack(theta):
    """Split the flat parameter vector into [W1, b1, ..., W5, b5] (views)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAMS
    out, o = [], 0
    for s in _SHAPES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def features(h, freqs):
    """Fourier features of offsets h (n, 2) with frequencies (64, 2): (n, 128)."""
    h = np.asarray(h, dtype=np.float64)
    t = 2.0 * np.pi * ((h - 0.5) @ np.asarray(freqs, dtype=np.float64).T)
    return np.concatenate([np.sin(t), np.cos(t)], axis=1)


def forward(theta, freqs, h):
    """Network outputs y (n, 16) and the per-layer cache for the backward pass."""
    P = unpack(theta)
    a = features(h, freqs)
    cache = [a]
    for l in range(N_LAYERS):
        z = a @ P[2 * l].T + P[2 * l + 1]
        a = np.maximum(z, 0.0)
        cache.append(a)
    y = a @ P[2 * N_LAYERS].T + P[2 * N_LAYERS + 1]
    return y, cache


TABLE_SIDE = 32


def table_nodes(T=TABLE_SIDE):
    """Offsets (n, 2) of the table's nodes, node b (T+1) + a at (a/T, b/T)."""
    a = np.arange(T + 1, dtype=np.float64) / T
    hx, hy = np.meshgrid(a, a)               # hx varies along a row (a), hy down (b)
    return np.stack([hx.ravel(), hy.ravel()], axis=1)


def table_blend(Y, h, T=TABLE_SIDE):
    """Bilinear blend (n, m) of node values Y ((T+1)^2, m) at offsets h (n, 2)."""
    h = np.clip(np.asarray(h, dtype=np.float64), 0.0, 1.0) * T
    a = np.minimum(np.floor(h[:, 0]).astype(np.int64), T - 1)
    b = np.minimum(np.floor(h[:, 1]).astype(np.int64), T - 1)
    fu = (h[:, 0] - a)[:, None]
    fv = (h[:, 1] - b)[:, None]
    k = b * (T + 1) + a
    return ((1 - fu) * (1 - fv) * Y[k] + fu * (1 - fv) * Y[k + 1]
            + (1 - fu) * fv * Y[k + T + 1] + fu * fv * Y[k + T + 2])


def table_weights(theta, freqs, h):
    """The weights (n, 16) the rays take at offsets h: the network's outputs
    at the table's nodes, blended."""
    Y, _ = forward(theta, freqs, table_nodes())
    return table_blend(Y, h)


def weights_complex(y):
    """L_k = y_{2k} + i y_{2k+1}: (n, 8) complex."""
    return y[:, 0::2] + 1j * y[:, 1::2]


def predict(theta, freqs, h, D):
    """sum_k L_k(h) D_k for data D (n, 8) complex."""
    y, _ = forward(theta, freqs, h)
    return np.sum(weights_complex(y) * D, axis=1)


def loss_and_grad(theta, freqs, h, D, T):
    """Mean squared error of the prediction against T and its gradient with
    respect to the flat parameter vector (plain reverse-mode chain rule)."""
    P = unpack(theta)
    n = h.shape[0]
    y, cache = forward(theta, freqs, h)
    r = np.sum(weights_complex(y) * D, axis=1) - T
    loss = float(np.mean(np.abs(r) ** 2))
    # d loss / d y: for L = yr + i yi, d|r|^2/dyr = 2 Re(r conj(D)), d/dyi = 2 Im(r conj(D))
    g = r[:, None] * np.conj(D) * (2.0 / n)
    dy = np.empty((n, N_OUT))
    dy[:, 0::2] = g.real
    dy[:, 1::2] = g.imag
    grads = [None] * len(P)
    grads[2 * N_LAYERS] = dy.T @ cache[N_LAYERS]
    grads[2 * N_LAYERS + 1] = dy.sum(axis=0)
    da = dy @ P[2 * N_LAYERS]
    for l in range(N_LAYERS - 1, -1, -1):
        dz = da * (cache[l + 1] > 0.0)
        grads[2 * l] = dz.T @ cache[l]
        grads[2 * l + 1] = dz.sum(axis=0)
        da = dz @ P[2 * l]
    return loss, np.concatenate([gg.ravel() for gg in grads])


# ---------------------------------------------------------------------------
# Coarse squares: base interpolant and local data
# ---------------------------------------------------------------------------

def square_corners(x0, y0, sx, sy):
    """Corner positions (n, 4) complex, order lower-left, lower-right,
    upper-left, upper-right."""
    x0, y0 = np.asarray(x0, float), np.asarray(y0, float)
    return np.stack([x0 + 1j * y0, (x0 + sx) + 1j * y0, x0 + 1j * (y0 + sy),
                     (x0 + sx) + 1j * (y0 + sy)], axis=1)


def bilinear(h):
    hx, hy = h[:, 0], h[:, 1]
    return np.stack([(1 - hx) * (1 - hy), hx * (1 - hy), (1 - hx) * hy, hx * hy], axis=1)


def base_interp(zc, Ac, dAc, h, z):
    """I(z) = sum_c w_c(h) (A_c + A'_c (z - z_c)); arrays (n, 4) complex."""
    w = bilinear(np.asarray(h, float))
    return np.sum(w * (Ac + dAc * (np.asarray(z)[:, None] - zc)), axis=1)


def local_data(zc, Ac, dAc, sx, sy, tiny=1e-280):
    """(D (n, 8) complex, sigma (n,)) of the squares, as defined above."""
    zm = zc.mean(axis=1, keepdims=True)
    Am = Ac.mean(axis=1, keepdims=True)
    dAm = dAc.mean(axis=1, keepdims=True)
    s = 0.5 * (sx + sy)
    delta = (dAc - dAm) * s
    eps = Ac - Am - dAm * (zc - zm)
    sigma = np.maximum(np.max(np.maximum(np.abs(delta), np.abs(eps)), axis=1), tiny)
    D = np.concatenate([delta, eps], axis=1) / sigma[:, None]
    return D, sigma


def learned_value(theta, freqs, zc, Ac, dAc, sx, sy, h, z):
    """I(z) + sigma sum_k L_k(h) D_k, L from the blended table."""
    D, sigma = local_data(zc, Ac, dAc, sx, sy)
    L = weights_complex(table_weights(theta, freqs, h))
    return base_interp(zc, Ac, dAc, h, z) + sigma * np.sum(L * D, axis=1)


# ---------------------------------------------------------------------------
# Rays with the learned interpolant (reference for the GPU path)
# ---------------------------------------------------------------------------

def _pixel(g, b1, b2):
    """Source pixel of beta (row-major, -1 off the map), as in O-1."""
    dpix = g.source_side / g.npix
    ix = np.floor((b1 + 0.5 * g.source_side) / dpix)
    iy = np.floor((b2 + 0.5 * g.source_side) / dpix)
    ok = (ix >= 0) & (ix < g.npix) & (iy >= 0) & (iy < g.npix)
    return np.where(ok, iy * g.npix + ix, -1).astype(np.int64)


def ray_squares(g, qc, ray_ids):
    """Ray positions, cells and squares: the coarse grid splits [a1, a2] into
    n1x*qc columns and the ray sits at the centre of its ray cell, so its
    column is floor((i + 1/2) n1x qc / nx), in integers."""
    r = np.asarray(ray_ids, dtype=np.int64)
    i, j = r % g.nx, r // g.nx
    gxc = ((2 * i + 1) * g.n1x * qc) // (2 * g.nx)
    gyc = ((2 * j + 1) * g.n1y * qc) // (2 * g.ny)
    t1 = g.a1 + (i + 0.5) * ((g.a2 - g.a1) / g.nx)
    t2 = g.b1 + (j + 0.5) * ((g.b2 - g.b1) / g.ny)
    return t1, t2, gxc, gyc


def learned_rays(g, lenses, cell_start, perm, qc, freqs, theta, ray_ids, threads=0):
    """alpha1, alpha2 and pixel of rays under the learned interpolant, with the
    network in FP64.  The near lenses, the macro term and the non-analytic part
    of the sheet are those of the direct definition, so
        alpha_learned = alpha_O1 + conj(A_learned(z) - A(z)),
    A the exact distant field of the ray's cell (orc_far_point)."""
    from .core import alpha_points, far_point
    t1, t2, gxc, gyc = ray_squares(g, qc, ray_ids)
    cx, cy = gxc // qc, gyc // qc
    sx = (g.a2 - g.a1) / (g.n1x * qc)
    sy = (g.b2 - g.b1) / (g.n1y * qc)
    X0, X1 = g.a1 + gxc * sx, g.a1 + (gxc + 1) * sx
    Y0, Y1 = g.b1 + gyc * sy, g.b1 + (gyc + 1) * sy
    n = t1.size
    px = np.stack([X0, X1, X0, X1], axis=1).ravel()
    py = np.stack([Y0, Y0, Y1, Y1], axis=1).ravel()
    Ac, dAc = far_point(g, lenses, cell_start, perm, np.repeat(cx, 4), np.repeat(cy, 4), px, py,
                        threads)
    Ac, dAc = Ac.reshape(n, 4), dAc.reshape(n, 4)
    zc = (px + 1j * py).reshape(n, 4)
    A, _ = far_point(g, lenses, cell_start, perm, cx, cy, t1, t2, threads)
    h = np.stack([(t1 - X0) / sx, (t2 - Y0) / sy], axis=1)
    Al = learned_value(theta, freqs, zc, Ac, dAc, sx, sy, h, t1 + 1j * t2)
    a1, a2, _ = alpha_points(g, lenses, t1, t2)
    d = Al - A
    a1 = a1 + d.real
    a2 = a2 - d.imag
    return a1, a2, _pixel(g, t1 - a1, t2 - a2)
