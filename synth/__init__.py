"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the tests, the oracle runs and the benchmark.  It
holds geometry and data generation only (curves, panels, quadrature nodes,
densities, sources, targets) and none of the potential-evaluation method's
arithmetic.

Recipes (Section 6 of the paper for the curve family, eq. (bound_curve)):
  * boundary curves gamma(t) = c + s (r0 + a cos(l1 t + b1) + b sin(l2 t + b2))
    exp(i (t + 0.1 sin(l3 t))), t in [0, 2 pi), counter-clockwise;
  * M panels of equal parameter length, 16 Gauss-Legendre nodes each
    (Section 3.2), exact normals (outward), curvature and weights;
  * volume: cut-cell quadrature on a background grid of equilateral
    triangles of side dx (Section 3.1) with a symmetric 6-point rule of
    degree 4 per triangle; cut triangles are clipped at the boundary
    crossings of their edges and fan-triangulated, and the sub-triangle on
    the boundary chord is made curved (its chord replaced by the quadratic
    through the two crossings and the boundary point between them), so
    that every node lies inside the body;  or, for accuracy studies, a
    spectrally accurate polar rule on star-shaped bodies;
  * densities: sum_{k<=8} a_k cos(k t) + b_k sin(k t), a_k, b_k ~ N(0,1)/max(1,k)^2;
  * sources: f = sum of 4 Gaussians of width 0.2 with N(0,1) amplitudes.
Random streams: np.random.default_rng(SeedSequence([config, stream])) with
stream 0 geometry, 1 density, 2 source, 3 targets, 4 arrivals.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field

import numpy as np

NGL = 16
STREAM_GEOMETRY, STREAM_DENSITY, STREAM_SOURCE, STREAM_TARGETS, STREAM_ARRIVALS = range(5)


def rng(config: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(config), int(stream)]))


# --------------------------------------------------------------------------
# Curves
# --------------------------------------------------------------------------
@dataclass
class Curve:
    """One closed curve of the paper's family, scaled by s and shifted by c."""
    r0: float = 1.0
    a: float = 0.0
    b: float = 0.0
    l1: int = 0
    l2: int = 0
    l3: int = 0
    b1: float = 0.0
    b2: float = 0.0
    s: float = 1.0
    cx: float = 0.0
    cy: float = 0.0

    def radius(self, t, d=0):
        R = [self.r0 + self.a * np.cos(self.l1 * t + self.b1) + self.b * np.sin(self.l2 * t + self.b2),
             -self.a * self.l1 * np.sin(self.l1 * t + self.b1) + self.b * self.l2 * np.cos(self.l2 * t + self.b2),
             -self.a * self.l1 ** 2 * np.cos(self.l1 * t + self.b1) - self.b * self.l2 ** 2 * np.sin(self.l2 * t + self.b2)]
        return R[d]

    def angle(self, t, d=0):
        th = [t + 0.1 * np.sin(self.l3 * t),
              1.0 + 0.1 * self.l3 * np.cos(self.l3 * t),
              -0.1 * self.l3 ** 2 * np.sin(self.l3 * t)]
        return th[d]

    def eval(self, t):
        """gamma, gamma', gamma'' as complex arrays."""
        R, R1, R2 = (self.radius(t, d) for d in range(3))
        th, th1, th2 = (self.angle(t, d) for d in range(3))
        e = np.exp(1j * th)
        g = self.s * R * e + (self.cx + 1j * self.cy)
        g1 = self.s * (R1 + 1j * R * th1) * e
        g2 = self.s * (R2 - R * th1 ** 2 + 1j * (2 * R1 * th1 + R * th2)) * e
        return g, g1, g2

    def inside(self, x, y):
        """Point-in-body test: invert the polar angle, compare radii."""
        dx = (np.asarray(x) - self.cx) / self.s
        dy = (np.asarray(y) - self.cy) / self.s
        phi = np.mod(np.arctan2(dy, dx), 2 * np.pi)
        t = phi.copy()
        if self.l3 != 0:
            for _ in range(30):
                t = t - (self.angle(t) - phi) / self.angle(t, 1)
        return np.hypot(dx, dy) < self.radius(t)

    def perimeter(self, n=4096):
        t = np.arange(n) * (2 * np.pi / n)
        return float(np.sum(np.abs(self.eval(t)[1])) * 2 * np.pi / n)

    def area(self, n=4096):
        t = np.arange(n) * (2 * np.pi / n)
        g, g1, _ = self.eval(t)
        return float(0.5 * np.sum((g.real * g1.imag - g.imag * g1.real)) * 2 * np.pi / n)

    def rmax(self):
        return self.s * (self.r0 + abs(self.a) + abs(self.b))


@functools.lru_cache(maxsize=None)
def gauss_legendre(n: int = NGL):
    return np.polynomial.legendre.leggauss(n)


def discretize(curves, panels):
    """Composite Gauss-Legendre discretisation of a list of curves.

    Returns a dict of panel-contiguous arrays: x, y, nx, ny (outward unit
    normal), w (weights, parameter speed included), kappa (signed curvature,
    positive on convex parts), t (curve parameter), curve (index),
    panel_prev, panel_next (cyclic within each curve), curve_panel_ofs.
    """
    if isinstance(panels, int):
        panels = [panels] * len(curves)
    tg, wg = gauss_legendre(NGL)
    out = {k: [] for k in ("x", "y", "nx", "ny", "w", "kappa", "t", "curve", "sx", "sy")}
    prev, nxt, ofs = [], [], [0]
    p0 = 0
    for ci, (cv, M) in enumerate(zip(curves, panels)):
        edges = np.linspace(0.0, 2 * np.pi, M + 1)
        ta, tb = edges[:-1, None], edges[1:, None]
        t = 0.5 * (ta + tb) + 0.5 * (tb - ta) * tg[None, :]
        g, g1, g2 = cv.eval(t)
        sp = np.abs(g1)
        out["x"].append(g.real.ravel()); out["y"].append(g.imag.ravel())
        out["nx"].append((g1.imag / sp).ravel()); out["ny"].append((-g1.real / sp).ravel())
        out["w"].append((0.5 * (tb - ta) * wg[None, :] * sp).ravel())
        out["kappa"].append(((g1.real * g2.imag - g1.imag * g2.real) / sp ** 3).ravel())
        out["t"].append(t.ravel()); out["curve"].append(np.full(t.size, ci))
        out["sx"].append((g1.real / sp).ravel()); out["sy"].append((g1.imag / sp).ravel())
        idx = np.arange(M)
        prev.append(p0 + (idx - 1) % M); nxt.append(p0 + (idx + 1) % M)
        p0 += M
        ofs.append(p0)
    b = {k: np.concatenate(v) for k, v in out.items()}
    b["panel_prev"] = np.concatenate(prev).astype(np.int64)
    b["panel_next"] = np.concatenate(nxt).astype(np.int64)
    b["curve_panel_ofs"] = np.array(ofs, dtype=np.int64)
    return b


def inside_any(curves, x, y):
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    m = np.zeros(np.shape(x), dtype=bool)
    for cv in curves:
        r = cv.rmax()
        sel = (np.abs(x - cv.cx) <= r) & (np.abs(y - cv.cy) <= r)
        if sel.any():
            m[sel] |= cv.inside(x[sel], y[sel])
    return m


# --------------------------------------------------------------------------
# Triangle rule: symmetric 6 points, degree 4, from the moment equations
# --------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def triangle_rule6():
    """Barycentric nodes (6,3) and weights (6,) summing to 1 (unit area).

    Two orbits of type (a, a, 1-2a) with weights w1, w2; the four unknowns
    solve the moment equations for the S3-invariant monomials up to degree
    4, evaluated exactly on the reference triangle.
    """
    from scipy.optimize import fsolve

    def moment(i, j):  # int over ref triangle (area 1/2) of x^i y^j, normalised by area
        return 2.0 * math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)

    monos = [(0, 0), (2, 0), (1, 1), (3, 0), (2, 1), (4, 0), (2, 2), (3, 1)]

    def pts(a):
        return np.array([[a, a], [a, 1 - 2 * a], [1 - 2 * a, a]])

    def eqs(v):
        a1, w1, a2, w2 = v
        P1, P2 = pts(a1), pts(a2)
        r = []
        for (i, j) in [(0, 0), (2, 0), (3, 0), (4, 0)]:
            q = w1 * np.sum(P1[:, 0] ** i * P1[:, 1] ** j) + w2 * np.sum(P2[:, 0] ** i * P2[:, 1] ** j)
            r.append(q - moment(i, j))
        return r

    a1, w1, a2, w2 = fsolve(eqs, [0.44, 0.22, 0.09, 0.11], xtol=1e-13)
    P = np.vstack([pts(a1), pts(a2)])
    W = np.array([w1] * 3 + [w2] * 3)
    for (i, j) in monos:
        assert abs(np.sum(W * P[:, 0] ** i * P[:, 1] ** j) - moment(i, j)) < 1e-13
    bary = np.column_stack([1 - P[:, 0] - P[:, 1], P[:, 0], P[:, 1]])
    return bary, W


def _tri_nodes(A, B, Cc):
    """6-point rule on triangles given vertex arrays (n,2). Returns x, y, w."""
    bary, W = triangle_rule6()
    X = bary[:, 0][None, :] * A[:, None, 0] + bary[:, 1][None, :] * B[:, None, 0] + bary[:, 2][None, :] * Cc[:, None, 0]
    Y = bary[:, 0][None, :] * A[:, None, 1] + bary[:, 1][None, :] * B[:, None, 1] + bary[:, 2][None, :] * Cc[:, None, 1]
    area = 0.5 * np.abs((B[:, 0] - A[:, 0]) * (Cc[:, 1] - A[:, 1]) - (Cc[:, 0] - A[:, 0]) * (B[:, 1] - A[:, 1]))
    Wt = area[:, None] * W[None, :]
    return X.ravel(), Y.ravel(), Wt.ravel()


def _tri_nodes_curved(A, B, Cc, M):
    """6-point rule on triangles whose edge B-C is replaced by the quadratic
    Q(s) through B, M, C (s in [0, 1]) and which are filled by the segments
    from A to Q (a blending map): x(l) = A + m (Q(s) - A) with m = lB + lC,
    s = lC/m, i.e. x = lA A + lB B + lC C + 4 lB lC/(lB + lC) (M - (B + C)/2).
    Every node lies on a segment from A to the curved edge, so the cell
    follows the boundary even when it is a sliver."""
    bary, W = triangle_rule6()
    d = M - 0.5 * (B + Cc)                                        # (n, 2)
    lA, lB, lC = bary[:, 0][None, :], bary[:, 1][None, :], bary[:, 2][None, :]
    m = lB + lC
    g = 4 * lB * lC / m
    X = lA * A[:, None, 0] + lB * B[:, None, 0] + lC * Cc[:, None, 0] + g * d[:, None, 0]
    Y = lA * A[:, None, 1] + lB * B[:, None, 1] + lC * Cc[:, None, 1] + g * d[:, None, 1]
    # Jacobian in (lB, lC): d g/d lB = 4 (lC/m)^2, d g/d lC = 4 (lB/m)^2
    gB, gC = 4 * (lC / m) ** 2, 4 * (lB / m) ** 2
    j11 = (B[:, None, 0] - A[:, None, 0]) + gB * d[:, None, 0]
    j21 = (B[:, None, 1] - A[:, None, 1]) + gB * d[:, None, 1]
    j12 = (Cc[:, None, 0] - A[:, None, 0]) + gC * d[:, None, 0]
    j22 = (Cc[:, None, 1] - A[:, None, 1]) + gC * d[:, None, 1]
    Wt = 0.5 * np.abs(j11 * j22 - j12 * j21) * W[None, :]
    return X.ravel(), Y.ravel(), Wt.ravel()


def _boundary_midpoints(curves, c1, c2, iters=48):
    """Point of the boundary on the perpendicular bisector of each chord
    c1-c2 (bisection on the inside test within half a chord length of the
    chord); the chord midpoint where no crossing is bracketed."""
    M = 0.5 * (c1 + c2)
    t = c2 - c1
    L = np.hypot(t[:, 0], t[:, 1])
    n = np.stack([-t[:, 1], t[:, 0]], -1) / np.maximum(L, 1e-300)[:, None]
    pa = M - 0.5 * L[:, None] * n
    pb = M + 0.5 * L[:, None] * n
    ia = inside_any(curves, pa[:, 0], pa[:, 1])
    ib = inside_any(curves, pb[:, 0], pb[:, 1])
    ok = ia != ib
    lo = np.where(ia[:, None], pa, pb)      # inside end
    hi = np.where(ia[:, None], pb, pa)      # outside end
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        im = inside_any(curves, mid[:, 0], mid[:, 1])
        lo = np.where(im[:, None], mid, lo)
        hi = np.where(im[:, None], hi, mid)
    return np.where(ok[:, None], 0.5 * (lo + hi), M)


def _edge_crossings(curves, ax, ay, ai, bx, by):
    """Boundary crossing on each edge a-b with exactly one end inside (ai:
    whether a is inside), by bisection on the inside test."""
    lx = np.where(ai, ax, bx); ly = np.where(ai, ay, by)
    hx = np.where(ai, bx, ax); hy = np.where(ai, by, ay)
    for _ in range(48):
        mx, my = 0.5 * (lx + hx), 0.5 * (ly + hy)
        im = inside_any(curves, mx, my)
        lx = np.where(im, mx, lx); ly = np.where(im, my, ly)
        hx = np.where(im, hx, mx); hy = np.where(im, hy, my)
    return 0.5 * (lx + hx), 0.5 * (ly + hy)


def _cut_cells(curves, CX, CY, CI):
    """Nodes of cut triangles (vertex arrays (n, 3), inside flags (n, 3)):
    the polygon inside the boundary chord, fan-triangulated from its first
    vertex, with the sub-triangle on the chord curved.  Returns x, y, w of
    shape (n, k) with k = 12 (unused slots weight 0)."""
    nc = len(CX)
    pts = np.zeros((nc, 6, 2))
    keep = np.zeros((nc, 6), dtype=bool)
    crossing = np.zeros((nc, 6), dtype=bool)
    for e in range(3):
        a, b = e, (e + 1) % 3
        pts[:, 2 * e, 0], pts[:, 2 * e, 1] = CX[:, a], CY[:, a]
        keep[:, 2 * e] = CI[:, a]
        cross = CI[:, a] != CI[:, b]
        idx = np.nonzero(cross)[0]
        px, py = _edge_crossings(curves, CX[idx, a], CY[idx, a], CI[idx, a], CX[idx, b], CY[idx, b])
        pts[idx, 2 * e + 1, 0] = px
        pts[idx, 2 * e + 1, 1] = py
        keep[:, 2 * e + 1] = cross
        crossing[:, 2 * e + 1] = cross
    # kept points in cyclic order (3 or 4 of them; the two crossings are
    # adjacent in the cycle and form the boundary chord)
    order = np.argsort(~keep, axis=1, kind="stable")
    P = np.take_along_axis(pts, order[:, :, None], axis=1)
    X_ = np.take_along_axis(crossing, order, axis=1)
    cntp = keep.sum(1)
    ar = np.arange(nc)
    k0 = np.full(nc, -1)
    for k in range(3, -1, -1):
        kn = (k + 1) % cntp
        isk = (k < cntp) & X_[ar, np.minimum(k, 5)] & X_[ar, kn]
        k0 = np.where(isk, k, k0)
    assert np.all(k0 >= 0)
    c1 = P[ar, k0]
    c2 = P[ar, (k0 + 1) % cntp]
    Mb = _boundary_midpoints(curves, c1, c2)
    # fan from P0: (P0, P1, P2) and, for 4-gons, (P0, P2, P3); the chord
    # (P_k, P_k+1) lies in the first for k in {0, 1} (3-gons: always), in the
    # second for k in {2, 3}; opposite vertex of the chord in its triangle
    tri3 = cntp == 3
    first = tri3 | (k0 <= 1)
    opp = np.where(tri3, (k0 + 2) % 3, np.where(k0 == 0, 2, np.where(k0 == 1, 0, np.where(k0 == 2, 0, 2))))
    x, y, w = (a.reshape(nc, 6) for a in _tri_nodes_curved(P[ar, opp], c1, c2, Mb))
    X = np.zeros((nc, 12)); Y = np.zeros((nc, 12)); Wt = np.zeros((nc, 12))
    X[:, :6], Y[:, :6], Wt[:, :6] = x, y, w
    # the straight other triangle of a 4-gon
    q4 = ~tri3
    A2 = np.where((q4 & ~first)[:, None], P[:, 0], P[:, 0])
    B2 = np.where((q4 & ~first)[:, None], P[:, 1], P[:, 2])
    C2 = np.where((q4 & ~first)[:, None], P[:, 2], P[:, 3])
    if q4.any():
        x, y, w = (a.reshape(-1, 6) for a in _tri_nodes(A2[q4], B2[q4], C2[q4]))
        X[q4, 6:], Y[q4, 6:], Wt[q4, 6:] = x, y, w
        # unused slots of 3-gons sit on the first node with weight 0
    X[~q4, 6:] = X[~q4, :1]; Y[~q4, 6:] = Y[~q4, :1]
    return X, Y, Wt


def cut_cell_volume(curves, dx, box=None, max_depth=4):
    """Cut-cell quadrature of the union of the curves' interiors.

    Background grid of equilateral triangles of side dx (Section 3.1).
    Triangles with all vertices inside are kept, those with all outside are
    dropped; cut triangles are clipped at the boundary crossings of their
    edges (located by bisection on the inside test) and fan-triangulated,
    and in the sub-triangle that carries the boundary chord that edge becomes
    the quadratic through the two crossings and the boundary point on the
    chord's perpendicular bisector (curved cut cells, mapped by blending
    towards the opposite vertex).  A triangle whose nodes are not all inside
    (the boundary crosses one of its edges more than once) is split into four
    and treated again, up to max_depth times, so that every node lies
    inside.
    """
    if box is None:
        xs = [c.cx for c in curves]; ys = [c.cy for c in curves]; rr = [c.rmax() for c in curves]
        box = (min(x - r for x, r in zip(xs, rr)) - dx, max(x + r for x, r in zip(xs, rr)) + dx,
               min(y - r for y, r in zip(ys, rr)) - dx, max(y + r for y, r in zip(ys, rr)) + dx)
    x0, x1, y0, y1 = box
    hy = dx * math.sqrt(3) / 2
    nx = int(math.ceil((x1 - x0) / dx)) + 2
    ny = int(math.ceil((y1 - y0) / hy)) + 1
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    VX = x0 + ii * dx + 0.5 * dx * (jj % 2)
    VY = y0 + jj * hy
    ins = inside_any(curves, VX, VY)
    tris = []
    for j in range(ny - 1):
        odd = j % 2
        i = np.arange(nx - 1)
        # two triangle orientations per row strip
        if odd == 0:
            t1 = ((j, i), (j, i + 1), (j + 1, i))
            t2 = ((j, i + 1), (j + 1, i + 1), (j + 1, i))
        else:
            t1 = ((j, i), (j, i + 1), (j + 1, i + 1))
            t2 = ((j, i), (j + 1, i + 1), (j + 1, i))
        for t in (t1, t2):
            tris.append(np.stack([np.stack([np.full_like(i, a[0]) if np.isscalar(a[0]) else a[0], a[1]], -1)
                                  for a in t], 1))
    T = np.concatenate(tris, 0)  # (nt, 3, 2) of (row, col)
    TX = VX[T[..., 0], T[..., 1]]; TY = VY[T[..., 0], T[..., 1]]; TI = ins[T[..., 0], T[..., 1]]
    xs, ys, ws = [], [], []
    for depth in range(max_depth + 1):
        cnt = TI.sum(1)
        full = np.nonzero(cnt == 3)[0]
        cut = np.nonzero((cnt > 0) & (cnt < 3))[0]
        # candidate nodes, (n, 12) per triangle (full triangles use 6 slots)
        NX = np.zeros((len(full) + len(cut), 12)); NY = np.zeros_like(NX); NW = np.zeros_like(NX)
        x, y, w = (a.reshape(-1, 6) for a in _tri_nodes(np.stack([TX[full, 0], TY[full, 0]], -1),
                                                       np.stack([TX[full, 1], TY[full, 1]], -1),
                                                       np.stack([TX[full, 2], TY[full, 2]], -1)))
        nf = len(full)
        NX[:nf, :6], NY[:nf, :6], NW[:nf, :6] = x, y, w
        NX[:nf, 6:], NY[:nf, 6:] = x[:, :1], y[:, :1]
        if len(cut):
            NX[nf:], NY[nf:], NW[nf:] = _cut_cells(curves, TX[cut], TY[cut], TI[cut])
        src = np.concatenate([full, cut])
        # triangles near the boundary: every node must be inside
        ok = np.ones(len(src), dtype=bool)
        near = np.ones(len(src), dtype=bool)
        near[:nf] = False
        if nf:
            # full triangles can hide a boundary bump only if a node of theirs
            # is outside; test those within one side length of a cut triangle
            # vertex cheaply by the inside test of all their nodes
            near[:nf] = True
        cand = np.nonzero(near)[0]
        inside_nodes = inside_any(curves, NX[cand].ravel(), NY[cand].ravel()).reshape(-1, 12)
        ok[cand] = inside_nodes.all(1)
        if depth == max_depth:
            ok[:] = True
        good = np.nonzero(ok)[0]
        xs.append(NX[good].ravel()); ys.append(NY[good].ravel()); ws.append(NW[good].ravel())
        bad = src[~ok]
        if len(bad) == 0:
            break
        # split the bad triangles into four at their edge midpoints
        ax, ay = TX[bad, 0], TY[bad, 0]; bx, by = TX[bad, 1], TY[bad, 1]; cx, cy = TX[bad, 2], TY[bad, 2]
        abx, aby = 0.5 * (ax + bx), 0.5 * (ay + by)
        bcx, bcy = 0.5 * (bx + cx), 0.5 * (by + cy)
        cax, cay = 0.5 * (cx + ax), 0.5 * (cy + ay)
        TX = np.concatenate([np.stack([ax, abx, cax], 1), np.stack([abx, bx, bcx], 1),
                             np.stack([cax, bcx, cx], 1), np.stack([abx, bcx, cax], 1)])
        TY = np.concatenate([np.stack([ay, aby, cay], 1), np.stack([aby, by, bcy], 1),
                             np.stack([cay, bcy, cy], 1), np.stack([aby, bcy, cay], 1)])
        TI = inside_any(curves, TX.ravel(), TY.ravel()).reshape(-1, 3)
    x = np.concatenate(xs); y = np.concatenate(ys); w = np.concatenate(ws)
    m = w > 0
    # unused slots have weight 0 six at a time: the kept nodes are in groups
    # of six, one triangle's 6-point rule each
    assert m.sum() % 6 == 0
    bary, W = triangle_rule6()
    rule = np.column_stack([bary[:, 1], bary[:, 2], W])     # (s, t, W) of the nodes of every group
    return {"x": x[m], "y": y[m], "w": w[m], "group": 6, "rule": rule}


def polar_volume(curve: Curve, n_rho: int, n_theta: int):
    """Spectrally accurate rule on a star-shaped body with angle(t) = t."""
    assert curve.l3 == 0
    tg, wg = gauss_legendre(n_rho)
    rho = 0.5 * (tg + 1); wr = 0.5 * wg
    th = np.arange(n_theta) * (2 * np.pi / n_theta)
    R = curve.s * curve.radius(th)
    X = curve.cx + rho[:, None] * R[None, :] * np.cos(th)[None, :]
    Y = curve.cy + rho[:, None] * R[None, :] * np.sin(th)[None, :]
    W = wr[:, None] * rho[:, None] * (R ** 2)[None, :] * (2 * np.pi / n_theta)
    return {"x": X.ravel(), "y": Y.ravel(), "w": W.ravel()}


# --------------------------------------------------------------------------
# Densities, sources, targets
# --------------------------------------------------------------------------
def fourier_density(t, curve_idx, g: np.random.Generator, n_curves: int, kmax: int = 8):
    k = np.arange(kmax + 1)
    scale = 1.0 / np.maximum(1, k) ** 2
    out = np.zeros_like(t)
    for c in range(n_curves):
        a = g.standard_normal(kmax + 1) * scale
        b = g.standard_normal(kmax + 1) * scale
        m = curve_idx == c
        out[m] = (a[None, :] * np.cos(np.outer(t[m], k)) + b[None, :] * np.sin(np.outer(t[m], k))).sum(1)
    return out


@dataclass
class GaussSource:
    cx: np.ndarray
    cy: np.ndarray
    amp: np.ndarray
    width: float = 0.2

    def __call__(self, x, y):
        s = 2 * self.width ** 2
        out = np.zeros(np.broadcast(x, y).shape)
        for cx, cy, a in zip(self.cx, self.cy, self.amp):
            out += a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / s)
        return out

    def jet(self, x, y):
        """[6, n]: f, f_x, f_y, f_xx, f_xy, f_yy at the points (analytic)."""
        s = 2 * self.width ** 2
        x, y = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float))
        out = np.zeros((6,) + x.shape)
        for cx, cy, a in zip(self.cx, self.cy, self.amp):
            dx, dy = x - cx, y - cy
            g = a * np.exp(-(dx * dx + dy * dy) / s)
            out[0] += g
            out[1] += -2 * dx / s * g
            out[2] += -2 * dy / s * g
            out[3] += (4 * dx * dx / s ** 2 - 2 / s) * g
            out[4] += 4 * dx * dy / s ** 2 * g
            out[5] += (4 * dy * dy / s ** 2 - 2 / s) * g
        return out


def gauss_source(g: np.random.Generator, centers_x, centers_y, width=0.2):
    return GaussSource(np.asarray(centers_x, float), np.asarray(centers_y, float),
                       g.standard_normal(len(centers_x)), width)


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    curves: list
    boundary: dict
    volume: dict
    tx: np.ndarray
    ty: np.ndarray
    inside: np.ndarray
    sigma: np.ndarray
    mu: np.ndarray
    f_vol: np.ndarray
    f_trg: np.ndarray          # f at off-surface targets then at boundary nodes
    alphas: tuple
    tol: float
    dx: float
    meta: dict = field(default_factory=dict)

    @property
    def n_b(self):
        return len(self.boundary["x"])

    @property
    def n_v(self):
        return len(self.volume["x"])

    @property
    def n_t(self):
        return len(self.tx)


def _densities_and_sources(cfg, curves, bnd, vol, tx, ty, src_centers):
    gd = rng(cfg, STREAM_DENSITY)
    sigma = fourier_density(bnd["t"], bnd["curve"], gd, len(curves))
    mu = fourier_density(bnd["t"], bnd["curve"], gd, len(curves))
    gs = rng(cfg, STREAM_SOURCE)
    fsrc = gauss_source(gs, *src_centers)
    f_vol = fsrc(vol["x"], vol["y"])
    f_trg = np.concatenate([fsrc(tx, ty), fsrc(bnd["x"], bnd["y"])])
    return sigma, mu, f_vol, f_trg, fsrc


def config0(n_panels=32, dx=0.1, grid=64):
    """Starfish r(t) = 1 + 0.3 cos 5t, 32 panels x 16 nodes, cut-cell volume
    on a background grid of side 0.1, 64x64 target grid on [-1.5,1.5]^2."""
    cfg = 0
    curves = [Curve(r0=1.0, a=0.3, l1=5)]
    bnd = discretize(curves, n_panels)
    vol = cut_cell_volume(curves, dx)
    g1 = np.linspace(-1.5, 1.5, grid)
    TX, TY = np.meshgrid(g1, g1, indexing="xy")
    tx, ty = TX.ravel(), TY.ravel()
    ins = inside_any(curves, tx, ty)
    gc = rng(cfg, STREAM_SOURCE)
    ang = gc.uniform(0, 2 * np.pi, 4); rad = 0.5 * np.sqrt(gc.uniform(0, 1, 4))
    sigma, mu, f_vol, f_trg, fsrc = _densities_and_sources(
        cfg, curves, bnd, vol, tx, ty, (rad * np.cos(ang), rad * np.sin(ang)))
    return Workload("starfish-512b-64x64", curves, bnd, vol, tx, ty, ins, sigma, mu, f_vol, f_trg,
                    (10.0,), 1e-10, dx, {"fsrc": fsrc})


def min_curvature_radius(curve: Curve, n=4096):
    t = np.arange(n) * (2 * np.pi / n)
    _, g1, g2 = curve.eval(t)
    k = np.abs(g1.real * g2.imag - g1.imag * g2.real) / np.abs(g1) ** 3
    return float(1.0 / k.max())


def random_bodies(cfg, n_bodies, rmin=0.05, rmax=0.2, box=1.0, gap=0.05, rcurv_min=0.02):
    """Non-overlapping seeded starfish bodies.  The arm amplitude drawn in
    [0.1, 0.3] is shrunk until the smallest radius of curvature is at least
    rcurv_min, so that targets near the boundary have a unique closest
    point (the assumption of Section 4.1)."""
    g = rng(cfg, STREAM_GEOMETRY)
    curves = []
    tries = 0
    while len(curves) < n_bodies:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place bodies")
        s = g.uniform(rmin, rmax); m = int(g.integers(3, 8)); a = g.uniform(0.1, 0.3)
        ph = g.uniform(0, 2 * np.pi)
        while min_curvature_radius(Curve(r0=1.0, a=a, l1=m, s=s)) < rcurv_min:
            a *= 0.9
        R = s * (1 + a)
        cx, cy = g.uniform(-box + R, box - R, 2)
        ok = all(math.hypot(cx - c.cx, cy - c.cy) > R + c.rmax() + gap for c in curves)
        if ok:
            curves.append(Curve(r0=1.0, a=a, l1=m, b1=ph, s=s, cx=cx, cy=cy))
    return curves


def multibody(cfg=1, n_bodies=10, n_boundary=16384, n_volume=1_000_000, n_targets=1_000_000,
              alphas=(1.0, 10.0, 100.0), tol=1e-10, box=1.0):
    """Seeded multi-body starfish workload (panels proportional to perimeter,
    cut-cell volume with dx set to reach n_volume nodes, targets uniform in
    the bodies' union)."""
    curves = random_bodies(cfg, n_bodies, box=box)
    per = np.array([c.perimeter() for c in curves])
    n_pan = n_boundary // NGL
    pan = np.maximum(8, np.floor(n_pan * per / per.sum()).astype(int))
    pan[np.argmax(per)] += n_pan - pan.sum()
    bnd = discretize(curves, list(pan))
    area = sum(c.area() for c in curves)
    dx = math.sqrt(6 * area / (math.sqrt(3) / 4 * n_volume))
    vol = cut_cell_volume(curves, dx)
    gt = rng(cfg, STREAM_TARGETS)
    # uniform in the union: sample per body proportional to area, reject
    areas = np.array([c.area() for c in curves])
    txs, tys = [], []
    need = n_targets
    while need > 0:
        which = gt.choice(len(curves), size=int(need * 1.6) + 16, p=areas / areas.sum())
        cxs = np.array([curves[k].cx for k in which]); cys = np.array([curves[k].cy for k in which])
        rr = np.array([curves[k].rmax() for k in which])
        px = cxs + gt.uniform(-1, 1, len(which)) * rr
        py = cys + gt.uniform(-1, 1, len(which)) * rr
        ok = np.zeros(len(which), bool)
        for k in range(len(curves)):
            m = which == k
            ok[m] = curves[k].inside(px[m], py[m])
        # the bounding squares have different areas: thin to equalise density
        keep_p = (rr / rr.max()) ** 2
        ok &= gt.uniform(0, 1, len(which)) < keep_p
        px, py = px[ok][:need], py[ok][:need]
        txs.append(px); tys.append(py); need -= len(px)
    tx, ty = np.concatenate(txs), np.concatenate(tys)
    ins = np.ones(len(tx), dtype=bool)
    gc = rng(cfg, STREAM_SOURCE)
    ci = gc.choice(len(curves), 4)
    cxs = np.array([curves[k].cx for k in ci]); cys = np.array([curves[k].cy for k in ci])
    sigma, mu, f_vol, f_trg, fsrc = _densities_and_sources(cfg, curves, bnd, vol, tx, ty, (cxs, cys))
    return Workload(f"multibody{n_bodies}-{len(bnd['x'])}b-{len(vol['x'])}v-{len(tx)}t",
                    curves, bnd, vol, tx, ty, ins, sigma, mu, f_vol, f_trg, tuple(alphas), tol, dx,
                    {"fsrc": fsrc})
