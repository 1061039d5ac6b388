"""Dyadic levels of the volume potential (oracle).

TEST INFRASTRUCTURE ONLY: imported by tests/, never by the product package.
numpy plus the oracle's direct level sum (mhk_oracle.c); nothing is shared
with the library.

The paper splits the local part of the layer potentials in time, a
first-order expansion over [0, delta*] and the dyadic corrections over
[delta/4^j, delta/4^(j-1)] summed on locally bisected panels (Section 4.2),
and notes that the same telescoping applies to the volume potential, where
a level is a two-dimensional quadrature over the mesh.  With J volume
levels:

    V = V_H(delta) + sum_{j=1..J} V_j + V_L(delta*),  delta* = delta/4^J,
    V_j(x) = sum_q w_q f(y_q) K_j^S(|x - y_q|),

K_j^S the single-layer difference kernel of level j (eq. (diffker_s); the
volume and single-layer kernels are the same) and V_L(delta*) Lemma 4.8 /
Corollaries 4.10, 4.11 with delta* in place of delta.

The level-j quadrature (nodes y_q, weights w_q), from the volume rule whose
nodes come in groups of six per triangle:
  * the reference rule: points (s_i, t_i) on T0 = {s, t >= 0, s + t <= 1}
    with weights W_i summing to 1, node i of a group being the triangle's
    image of (s_i, t_i);
  * the triangle's map x(s, t): the quadratic in (s, t) through its six
    nodes (exact for the straight triangles);
  * T0 split into 4^j congruent triangles (n = 2^j segments per side: the
    upright ones with corner (a, b)/n, a + b <= n - 1, and the inverted ones
    with corner (a + 1, b + 1)/n, a + b <= n - 2), each carrying the rule
    mapped onto it;
  * node y = x(s, t) at a mapped point, weight W_i |det Dx(s, t)| / (2 4^j);
  * f(y) from the quadratic of oracle.fjets fitted to the six nodal values
    of the node's own triangle; for the slivers that rule excludes, the
    quadratic of the triangle holding the nearest usable volume node.
"""
from __future__ import annotations

import numpy as np

import oracle as O
from oracle import fjets

GROUP = 6


def map_coefficients(vx, vy, rule):
    """Coefficients (ntri, 6) of x(s, t) and y(s, t) in the monomials
    1, s, t, s^2, s t, t^2, through the six nodes of each group."""
    s, t = rule[:, 0], rule[:, 1]
    R = np.stack([np.ones(6), s, t, s * s, s * t, t * t], 1)
    X = np.asarray(vx, np.float64).reshape(-1, GROUP)
    Y = np.asarray(vy, np.float64).reshape(-1, GROUP)
    return np.linalg.solve(R, X.T).T, np.linalg.solve(R, Y.T).T


def sub_points(j, rule):
    """Mapped rule points on the 4^j sub-triangles of T0: (m, 2) and the
    weights W_i / 4^j."""
    n = 1 << j
    s, t, W = rule[:, 0], rule[:, 1], rule[:, 2]
    pts, wts = [], []
    for b in range(n):
        for a in range(n - b):
            pts.append(np.stack([(a + s) / n, (b + t) / n], 1))
            wts.append(W / n ** 2)
    for b in range(n - 1):
        for a in range(n - 1 - b):
            pts.append(np.stack([(a + 1 - s) / n, (b + 1 - t) / n], 1))
            wts.append(W / n ** 2)
    return np.concatenate(pts), np.concatenate(wts)


def level_nodes(volume, rule, j):
    """Positions and weights of the level-j volume quadrature."""
    ax, ay = map_coefficients(volume["x"], volume["y"], rule)
    P, Wt = sub_points(j, rule)
    s, t = P[:, 0], P[:, 1]
    M = np.stack([np.ones_like(s), s, t, s * s, s * t, t * t], 1)          # (m, 6)
    Ms = np.stack([0 * s, np.ones_like(s), 0 * s, 2 * s, t, 0 * s], 1)       # d/ds
    Mt = np.stack([0 * s, 0 * s, np.ones_like(s), 0 * s, s, 2 * t], 1)      # d/dt
    x = ax @ M.T
    y = ay @ M.T
    det = (ax @ Ms.T) * (ay @ Mt.T) - (ax @ Mt.T) * (ay @ Ms.T)
    w = np.abs(det) * Wt[None, :] / 2.0
    return x.ravel(), y.ravel(), w.ravel()


def level_f(volume, f_vol, j, x, y):
    """f at the level-j nodes (x, y), in the order of level_nodes."""
    cen, h, thin, A = fjets.triangles(volume["x"], volume["y"])
    ntri = len(h)
    per_tri = len(x) // ntri
    parent = np.arange(len(x)) // per_tri
    usable = thin >= fjets.THIN_MIN
    c = np.zeros((ntri, GROUP))
    c[usable] = np.linalg.solve(A[usable], np.asarray(f_vol, np.float64).reshape(-1, GROUP)[usable][..., None])[..., 0]
    X = (x - cen[parent, 0]) / h[parent]
    Y = (y - cen[parent, 1]) / h[parent]
    cp = c[parent]
    f = cp[:, 0] + cp[:, 1] * X + cp[:, 2] * Y + cp[:, 3] * X * X + cp[:, 4] * X * Y + cp[:, 5] * Y * Y
    bad = np.nonzero(thin[parent] < fjets.THIN_MIN)[0]
    if len(bad):
        f[bad] = fjets.jets(volume["x"], volume["y"], f_vol, x[bad], y[bad])[0]
    return f


def levels(volume, rule, f_vol, alpha, delta, J, px, py):
    """sum_{j=1..J} V_j at the points (px, py) and the per-level values."""
    per = []
    for j in range(1, J + 1):
        x, y, w = level_nodes(volume, rule, j)
        f = level_f(volume, f_vol, j, x, y)
        per.append(O.level_sum_S(alpha, delta, j, x, y, w * f, px, py))
    return np.sum(per, 0), per


def volume_potential(w, alpha, delta, J, rule, f_trg, subset=None, order=1, f_jet=None):
    """V with J volume levels at the outputs of workload w (targets then
    boundary nodes; the subset of them): history at delta, levels, local
    part at delta / 4^J."""
    tx = np.concatenate([w.tx, w.boundary["x"]])
    ty = np.concatenate([w.ty, w.boundary["y"]])
    sel = np.arange(len(tx)) if subset is None else np.asarray(subset)
    kw = dict(volume=w.volume, targets=(w.tx, w.ty), inside=w.inside, on_surface=True, sigma=w.sigma, mu=w.mu,
              f_vol=w.f_vol, f_trg=f_trg, local_order=order, f_jet=f_jet)
    VH = O.Problem(alpha, delta, J, w.boundary, parts=O.PART_HISTORY, **kw).eval(subset)[2]
    VL = O.Problem(alpha, delta / 4 ** J, J, w.boundary, parts=O.PART_LOCAL, **kw).eval(subset)[2]
    lev, _ = levels(w.volume, rule, w.f_vol, alpha, delta, J, tx[sel], ty[sel])
    return VH + lev + VL
