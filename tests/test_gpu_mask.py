"""Inside mask computed by the plan when the caller passes none.

The mask decides which local expansions apply at a target (the sign rho of
the layer terms, Lemma 4.8 inside and its complement form outside), so a
plan with a wrong mask gives visibly different S, D, V at that target.  The
pins are the analytic point-in-body tests of the generated curves and, for
points a tiny distance off the curve between two boundary nodes (where the
polygon through the nodes puts about a third of them on the wrong side),
the side of the offset along the outward normal.  A plan built without a
mask must reproduce the plan built with the true mask; the two differ only
by the summation order of the spreading's LDS atomics."""
import numpy as np
import pytest

import synth
from helpers import small_multibody

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NGL = 16


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _near_points(curve, panels, eps_list, step=3):
    """Points gamma(t) +- eps n(t) midway between consecutive nodes (and
    between the end points and the first and last node) of every step-th
    panel of one curve: (x, y, inside)."""
    tg, _ = np.polynomial.legendre.leggauss(NGL)
    mids = np.concatenate([[0.5 * (-1 + tg[0])], 0.5 * (tg[:-1] + tg[1:]), [0.5 * (tg[-1] + 1)]])
    xs, ys, ins = [], [], []
    for p in range(0, panels, step):
        ta, tb = 2 * np.pi * p / panels, 2 * np.pi * (p + 1) / panels
        tc = 0.5 * (ta + tb) + 0.5 * (tb - ta) * mids
        g, g1, _ = curve.eval(tc)
        nx, ny = g1.imag / np.abs(g1), -g1.real / np.abs(g1)
        for eps in eps_list:
            for sg in (1.0, -1.0):
                xs.append(g.real + sg * eps * nx)
                ys.append(g.imag + sg * eps * ny)
                ins.append(np.full(len(tc), sg < 0))
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ins).astype(np.int8)


def _compare(bnd, vol, tx, ty, truth, f_fun, alpha=10.0, dx=None):
    import paper_2606_28865_amd as M
    X = np.concatenate([tx, bnd["x"]])
    Y = np.concatenate([ty, bnd["y"]])
    nb = len(bnd["x"])
    g = np.random.default_rng(7)
    sigma = np.cos(3 * np.arange(nb) / nb * 2 * np.pi) + 0.1 * g.standard_normal(nb)
    mu = np.sin(2 * np.arange(nb) / nb * 2 * np.pi) + 0.1 * g.standard_normal(nb)
    f_vol = f_fun(vol["x"], vol["y"])
    f_trg = f_fun(X, Y)
    outs = []
    for mask in (None, truth):
        kw = dict(alpha=alpha, tol=1e-10)
        if dx is not None:
            kw["dx"] = dx
        plan = M.Plan(M.make_params(**kw), bnd, vol, (tx, ty, mask), on_surface=True)
        outs.append([o.cpu().numpy().ravel() for o in plan.eval(_dev(sigma), _dev(mu), _dev(f_vol), _dev(f_trg))])
        plan.close()
    errs = []
    for a, b in zip(*outs):
        m = np.isfinite(b)
        assert np.array_equal(m, np.isfinite(a))
        errs.append(float(np.abs(a[m] - b[m]).max() / np.abs(b[m]).max()))
    return errs


def test_mask_config0_grid_and_near_curve():
    w = synth.config0()
    cv = w.curves[0]
    nx_, ny_, nin = _near_points(cv, 32, (1e-8, 1e-6, 1e-4, 1e-3))
    tx = np.concatenate([w.tx, nx_])
    ty = np.concatenate([w.ty, ny_])
    truth = np.concatenate([w.inside.astype(np.int8), nin])
    print(f"case computed mask config0: {len(w.tx)} grid targets, {len(nx_)} near the curve", flush=True)
    fsrc = w.meta["fsrc"]
    errs = _compare(w.boundary, w.volume, tx, ty, truth, lambda x, y: fsrc(x, y), dx=w.dx)
    print(f"computed vs true mask: S {errs[0]:.2e} D {errs[1]:.2e} V {errs[2]:.2e}", flush=True)
    assert max(errs) < 1e-12


def test_mask_multibody_box():
    w = small_multibody()
    g = np.random.default_rng(12)
    ux = g.uniform(-0.6, 0.6, 4000)
    uy = g.uniform(-0.6, 0.6, 4000)
    parts = [(ux, uy, synth.inside_any(w.curves, ux, uy).astype(np.int8))]
    ofs = w.boundary["curve_panel_ofs"]
    for c, cv in enumerate(w.curves):
        parts.append(_near_points(cv, int(ofs[c + 1] - ofs[c]), (1e-7, 1e-5), step=7))
    tx = np.concatenate([p[0] for p in parts])
    ty = np.concatenate([p[1] for p in parts])
    truth = np.concatenate([p[2] for p in parts])
    print(f"case computed mask 3-body box: {len(tx)} targets, {int(truth.sum())} inside", flush=True)
    fsrc = w.meta["fsrc"]
    errs = _compare(w.boundary, w.volume, tx, ty, truth, lambda x, y: fsrc(x, y), alpha=30.0, dx=w.dx)
    print(f"computed vs true mask: S {errs[0]:.2e} D {errs[1]:.2e} V {errs[2]:.2e}", flush=True)
    assert max(errs) < 1e-12
