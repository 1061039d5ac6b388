"""Checks of the seeded input generators (geometry and data only)."""
import math

import numpy as np
import pytest

import synth


def test_triangle_rule_degree4():
    bary, W = synth.triangle_rule6()
    assert W.sum() == pytest.approx(1.0, abs=1e-15)
    P = bary[:, 1:]
    for i in range(5):
        for j in range(5 - i):
            ex = 2.0 * math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
            assert np.sum(W * P[:, 0] ** i * P[:, 1] ** j) == pytest.approx(ex, abs=1e-14)


def test_starfish_discretisation():
    cv = synth.Curve(r0=1.0, a=0.3, l1=5)
    b = synth.discretize([cv], 32)
    assert len(b["x"]) == 512
    assert b["w"].sum() == pytest.approx(cv.perimeter(1 << 16), rel=1e-10)
    # area by the divergence theorem on the GL rule: 1/2 sum (x nx + y ny) w
    area = 0.5 * np.sum((b["x"] * b["nx"] + b["y"] * b["ny"]) * b["w"])
    assert area == pytest.approx(math.pi * (1 + 0.3 ** 2 / 2), rel=1e-10)
    # curvature integrates to 2 pi over a closed curve
    assert np.sum(b["kappa"] * b["w"]) == pytest.approx(2 * math.pi, rel=1e-10)


def test_cut_cell_volume_area_and_degree():
    cv = synth.Curve(r0=1.0, a=0.3, l1=5)
    v = synth.cut_cell_volume([cv], 0.05)
    area = math.pi * (1 + 0.3 ** 2 / 2)
    assert v["w"].sum() == pytest.approx(area, rel=2e-3)       # straight-edge cut cells
    assert np.all(v["w"] > 0)
    assert np.all(synth.inside_any([cv], v["x"], v["y"]) | (v["w"] < 1e-3))


def test_config0_shapes():
    w = synth.config0()
    assert w.n_b == 512 and w.n_t == 4096
    assert 4000 < w.n_v < 8000
    assert len(w.f_trg) == w.n_t + w.n_b
    assert w.inside.mean() == pytest.approx(w.curves[0].area() / 9.0, abs=0.02)


def test_random_bodies_separated_and_smooth():
    cs = synth.random_bodies(1, 10)
    for i, a in enumerate(cs):
        assert synth.min_curvature_radius(a) >= 0.02 - 1e-12
        for b in cs[:i]:
            assert math.hypot(a.cx - b.cx, a.cy - b.cy) > a.rmax() + b.rmax() + 0.05


def test_cut_cells_conform_to_the_boundary():
    """Curved cut cells: every node inside, and area and a smooth integral
    converging fast under refinement (against the polar rule)."""
    cv = [synth.Curve(r0=1.0, a=0.3, l1=5)]
    pv = synth.polar_volume(cv[0], 80, 400)
    f = lambda x, y: np.exp(0.5 * x) * np.cos(y)
    ref = (pv["w"] * f(pv["x"], pv["y"])).sum()
    errs = []
    for dx in (0.05, 0.0125):
        v = synth.cut_cell_volume(cv, dx)
        assert synth.inside_any(cv, v["x"], v["y"]).all()
        assert np.all(v["w"] > 0)
        errs.append(abs((v["w"] * f(v["x"], v["y"])).sum() - ref))
        assert abs(v["w"].sum() - cv[0].area()) < (2e-5 if dx > 0.02 else 2e-6)
    assert errs[1] < errs[0] / 4 and errs[1] < 2e-6, errs
