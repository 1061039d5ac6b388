"""Pins of the oracle's f-jet reconstruction from the volume quadrature
(CPU): exact for quadratic f, the expected orders for a smooth f under mesh
refinement, and the nearest-node rule against a k-d tree."""
import numpy as np

import synth
from oracle import fjets


def _mesh(dx):
    cv = synth.Curve(r0=1.0, a=0.3, l1=5)
    return synth.cut_cell_volume([cv], dx), cv


def _interior_points(cv, n, seed):
    g = np.random.default_rng(seed)
    p = g.uniform(-1.2, 1.2, size=(4 * n, 2))
    m = cv.inside(p[:, 0], p[:, 1])
    return p[m][:n]


def test_quadratic_is_reproduced():
    vol, cv = _mesh(0.1)
    c = [1.0, 2.0, -3.0, 0.5, -0.7, 0.25]
    f = lambda x, y: c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
    p = _interior_points(cv, 400, 1)
    J = fjets.jets(vol["x"], vol["y"], f(vol["x"], vol["y"]), p[:, 0], p[:, 1])
    x, y = p[:, 0], p[:, 1]
    exact = [f(x, y), c[1] + 2 * c[3] * x + c[4] * y, c[2] + c[4] * x + 2 * c[5] * y,
             np.full_like(x, 2 * c[3]), np.full_like(x, c[4]), np.full_like(x, 2 * c[5])]
    for k in range(6):
        assert np.abs(J[k] - exact[k]).max() < 1e-9 * max(1.0, np.abs(exact[k]).max()), k


def test_orders_for_a_gaussian():
    """f = exp(-|x - c|^2/s^2): value O(h^3), gradient O(h^2), Hessian O(h)
    at fixed interior points, h halved twice."""
    s, c = 0.4, (0.2, -0.1)
    def exact(x, y):
        dx, dy = x - c[0], y - c[1]
        e = np.exp(-(dx * dx + dy * dy) / s ** 2)
        fx, fy = -2 * dx / s ** 2 * e, -2 * dy / s ** 2 * e
        fxx = (4 * dx * dx / s ** 4 - 2 / s ** 2) * e
        fyy = (4 * dy * dy / s ** 4 - 2 / s ** 2) * e
        fxy = 4 * dx * dy / s ** 4 * e
        return [e, fx, fy, fxx, fxy, fyy]
    _, cv = _mesh(0.1)
    p = _interior_points(cv, 300, 2)
    errs = []
    for dx in (0.08, 0.04, 0.02):
        vol, _ = _mesh(dx)
        J = fjets.jets(vol["x"], vol["y"], exact(vol["x"], vol["y"])[0], p[:, 0], p[:, 1])
        ex = exact(p[:, 0], p[:, 1])
        errs.append([np.abs(J[0] - ex[0]).max(), max(np.abs(J[k] - ex[k]).max() for k in (1, 2)),
                     max(np.abs(J[k] - ex[k]).max() for k in (3, 4, 5))])
    errs = np.array(errs)
    # observed orders over the two halvings (the maximum over points is
    # noisy from one mesh to the next: which triangle holds the nearest
    # node changes): 3, 2 and 1 expected
    order = np.log2(errs[0] / errs[2]) / 2
    print(errs, order)
    assert order[0] > 2.6 and order[1] > 1.7 and order[2] > 0.85


def test_nearest_node_rule():
    from scipy.spatial import cKDTree
    vol, cv = _mesh(0.1)
    _, _, thin, _ = fjets.triangles(vol["x"], vol["y"])
    usable = np.nonzero(np.repeat(thin >= fjets.THIN_MIN, 6))[0]
    p = _interior_points(cv, 500, 3)
    got = fjets.nearest_usable_node(vol["x"], vol["y"], p[:, 0], p[:, 1])
    d, k = cKDTree(np.column_stack([vol["x"][usable], vol["y"][usable]])).query(p)
    dg = np.hypot(vol["x"][got] - p[:, 0], vol["y"][got] - p[:, 1])
    assert np.allclose(dg, d, rtol=0, atol=1e-15)
    assert np.isin(got, usable).all()
