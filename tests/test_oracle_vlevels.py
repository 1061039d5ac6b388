"""Pins of the oracle's dyadic volume levels (CPU): the level quadrature is
exact for polynomials of degree 4 on straight triangles (the reference
rule's degree), and each level of a Gaussian source matches its
whole-plane value, the time integral of the heat-smoothed Gaussian over
the level's interval, at points whose kernel does not reach the boundary."""
import numpy as np
from scipy import integrate

import oracle as O
import synth
from oracle import vlevels


def _rule():
    bary, W = synth.triangle_rule6()
    return np.column_stack([bary[:, 1], bary[:, 2], W])


def test_level_rule_exact_on_straight_triangles():
    g = np.random.default_rng(0)
    A = g.uniform(-1, 1, (20, 2)); B = A + g.uniform(0.1, 0.5, (20, 2)); C = A + g.uniform(-0.5, 0.1, (20, 2))
    x, y, w = synth._tri_nodes(A, B, C)
    vol = {"x": x, "y": y, "w": w, "group": 6}
    rule = _rule()
    polys = [lambda x, y: np.ones_like(x), lambda x, y: x * x * y, lambda x, y: x ** 4 - 2 * x * y ** 3 + y ** 2,
             lambda x, y: x ** 3 * y + 0.5 * y ** 4]
    for j in (1, 2, 3):
        qx, qy, qw = vlevels.level_nodes(vol, rule, j)
        assert len(qx) == 6 * 20 * 4 ** j
        for p in polys:
            coarse = np.sum(w * p(x, y))
            fine = np.sum(qw * p(qx, qy))
            assert abs(fine - coarse) < 1e-13 * max(1.0, abs(coarse)), (j, fine, coarse)


def test_levels_of_a_gaussian_match_whole_plane_values():
    # a disk of radius 0.6: the points lie within 0.2 of the source's centre,
    # so the boundary is 0.35 away, where K_1 is e^-30 of its peak and the
    # Gaussian e^-21 of its own
    cv = synth.Curve(r0=0.6)
    vol = synth.cut_cell_volume([cv], 0.05)
    alpha, delta, J = 10.0, 1e-3, 3
    s, c = 0.12, (0.05, -0.03)
    f = np.exp(-((vol["x"] - c[0]) ** 2 + (vol["y"] - c[1]) ** 2) / s ** 2)
    g = np.random.default_rng(1)
    r = 0.2 * np.sqrt(g.uniform(size=12)); th = g.uniform(0, 2 * np.pi, 12)
    px, py = c[0] + r * np.cos(th), c[1] + r * np.sin(th)
    _, per = vlevels.levels(vol, _rule(), f, alpha, delta, J, px, py)
    for j in range(1, J + 1):
        lo, hi = delta / 4 ** j, delta / 4 ** (j - 1)
        exact = np.array([integrate.quad(
            lambda t: np.exp(-alpha ** 2 * t) * s ** 2 / (s ** 2 + 4 * t)
            * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / (s ** 2 + 4 * t)), lo, hi, epsabs=0, epsrel=1e-12)[0]
            for x, y in zip(px, py)])
        err = np.abs(per[j - 1] - exact).max() / np.abs(exact).max()
        print(j, err)
        # quadrature of the level kernel and the quadratic reconstruction of
        # f at the refined nodes: a few 1e-5; a wrong interval, weight or
        # kernel would be off by O(1)
        assert err < 2e-4, (j, err)
