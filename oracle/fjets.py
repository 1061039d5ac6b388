"""f and its derivatives at targets from the volume quadrature (oracle).

TEST INFRASTRUCTURE ONLY: imported by tests/ and by the oracle's own
evaluation, never by the product package.  Plain numpy, FP64, written from
the definition below; it shares nothing with the library.

The volume potential's local part (Lemma 4.8 and Corollary 4.11) needs f
at the target x, and its second-order terms f's gradient and Hessian; the
volume quadrature (Section 3.1) carries f only at its nodes.  With the
nodes in consecutive groups of six per triangle (the 6-point rule of each
background or cut triangle), f near x is taken from the quadratic that
interpolates f at the six nodes of one triangle:

  * triangle of a group: centroid c of its six nodes, scale h = largest
    distance of a node from c, scaled coordinates (X, Y) = (x - c)/h;
  * shape measure: the smaller eigenvalue of the 2 x 2 matrix
    (1/6) sum over the nodes of (X, Y)^T (X, Y); triangles below THIN_MIN
    (slivers of the cut cells, whose six nodes are nearly collinear and
    make the quadratic ill-determined across them) are not used;
  * the triangle of x: the one holding the nearest node of a usable
    triangle (squared distance, ties to the lowest node index);
  * the quadratic q = c0 + c1 X + c2 Y + c3 X^2 + c4 X Y + c5 Y^2 through
    the six nodal values (a 6 x 6 linear solve), and at x: f = q,
    f_x = (c1 + 2 c3 X + c4 Y)/h, f_y = (c2 + c4 X + 2 c5 Y)/h,
    f_xx = 2 c3/h^2, f_xy = c4/h^2, f_yy = 2 c5/h^2.

It is exact for quadratic f; for smooth f the value errs by O(h^3), the
gradient by O(h^2) and the Hessian by O(h) (pinned in the tests).  Targets
that need f: those inside the domain and the boundary nodes (the exterior
volume term takes f at the closest boundary point from the latter).
"""
from __future__ import annotations

import numpy as np

GROUP = 6
THIN_MIN = 1e-3


def triangles(vx, vy):
    """Centroids (n, 2), scales (n,), shape measures (n,) and the 6 x 6
    matrices (n, 6, 6) of the node groups."""
    x = np.asarray(vx, np.float64).reshape(-1, GROUP)
    y = np.asarray(vy, np.float64).reshape(-1, GROUP)
    cx, cy = x.mean(1), y.mean(1)
    h = np.sqrt(((x - cx[:, None]) ** 2 + (y - cy[:, None]) ** 2).max(1))
    X = (x - cx[:, None]) / h[:, None]
    Y = (y - cy[:, None]) / h[:, None]
    a, b, c = (X * X).mean(1), (X * Y).mean(1), (Y * Y).mean(1)
    thin = 0.5 * (a + c) - np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    A = np.stack([np.ones_like(X), X, Y, X * X, X * Y, Y * Y], -1)
    return np.stack([cx, cy], 1), h, thin, A


def nearest_usable_node(vx, vy, px, py):
    """Index of the nearest node of a usable triangle to each (px, py), ties
    to the lowest index; brute force."""
    vx = np.asarray(vx, np.float64)
    vy = np.asarray(vy, np.float64)
    _, _, thin, _ = triangles(vx, vy)
    ok = np.repeat(thin >= THIN_MIN, GROUP)
    idx = np.nonzero(ok)[0]
    out = np.empty(len(px), np.int64)
    for s in range(0, len(px), 256):
        dx = np.asarray(px[s:s + 256])[:, None] - vx[None, idx]
        dy = np.asarray(py[s:s + 256])[:, None] - vy[None, idx]
        out[s:s + 256] = idx[np.argmin(dx * dx + dy * dy, axis=1)]   # argmin: first of equal minima
    return out


def jets(vx, vy, f_vol, px, py):
    """f, f_x, f_y, f_xx, f_xy, f_yy at the points (px, py): array (6, n)."""
    cen, h, thin, A = triangles(vx, vy)
    f6 = np.asarray(f_vol, np.float64).reshape(-1, GROUP)
    node = nearest_usable_node(vx, vy, px, py)
    t = node // GROUP
    c = np.linalg.solve(A[t], f6[t][..., None])[..., 0]                # (n, 6)
    X = (np.asarray(px) - cen[t, 0]) / h[t]
    Y = (np.asarray(py) - cen[t, 1]) / h[t]
    ht = h[t]
    return np.stack([c[:, 0] + c[:, 1] * X + c[:, 2] * Y + c[:, 3] * X * X + c[:, 4] * X * Y + c[:, 5] * Y * Y,
                     (c[:, 1] + 2 * c[:, 3] * X + c[:, 4] * Y) / ht,
                     (c[:, 2] + c[:, 4] * X + 2 * c[:, 5] * Y) / ht,
                     2 * c[:, 3] / ht ** 2, c[:, 4] / ht ** 2, 2 * c[:, 5] / ht ** 2])


def f_at_targets(volume, f_vol, tx, ty, inside, boundary=None, rows=1):
    """f_trg as the library reconstructs it: [rows][n_out] over the targets
    then (if boundary is given) the boundary nodes; rows 1 (f) or 6 (jets).
    Entries of exterior targets, which the local part never reads, are
    zero."""
    tx = np.asarray(tx, np.float64)
    ty = np.asarray(ty, np.float64)
    px, py = tx, ty
    need = np.asarray(inside).astype(bool)
    if boundary is not None:
        px = np.concatenate([tx, boundary["x"]])
        py = np.concatenate([ty, boundary["y"]])
        need = np.concatenate([need, np.ones(len(boundary["x"]), bool)])
    out = np.zeros((6, len(px)))
    sel = np.nonzero(need)[0]
    if len(sel):
        out[:, sel] = jets(volume["x"], volume["y"], f_vol, px[sel], py[sel])
    return out[:rows]
