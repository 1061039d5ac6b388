"""Pins of the boundary-integral-equation oracle (Section 3.2) against closed
forms and manufactured solutions.

* The Nystrom matrix on a circle against the exact spectrum of the
  double-layer operator (addition theorem of K_0: the interior and exterior
  limits of D[e^{in theta}] are aR I_n(aR) K_n'(aR) and aR I_n'(aR) K_n(aR)
  times e^{in theta}, a = alpha), converging as the panels are refined.
* The Dirichlet and Neumann solves for u a sum of K_0 sources outside the
  starfish (f = 0), against u itself at interior targets and on the
  boundary, converging in the number of panels; and a Dirichlet solve with a
  volume source, u = exp(ax + by), f = (alpha^2 - a^2 - b^2) u.
A wrong sign of the jump term, of the diagonal curvature term, a transposed
matrix or a dropped representation term fails at least one of these.
"""
import numpy as np
import pytest
import scipy.special as sp

import synth
from oracle import bie


def _spectrum_error(alpha, R, M):
    b = synth.discretize([synth.Curve(r0=R)], M)
    K = bie.nystrom_matrix(b, alpha)
    th = b["t"]
    z = alpha * R
    err = 0.0
    for n in range(0, 9):
        for c in (np.cos(n * th), np.sin(n * th)):
            if not np.any(c):
                continue
            lam_int = z * sp.iv(n, z) * sp.kvp(n, z)       # -1/2 + D on e^{in theta}
            lam_ext = z * sp.ivp(n, z) * sp.kv(n, z)       # +1/2 + D
            err = max(err, np.abs(-0.5 * c + K @ c - lam_int * c).max(), np.abs(0.5 * c + K @ c - lam_ext * c).max())
    return err


@pytest.mark.parametrize("alpha", [1.0, 10.0])
def test_nystrom_circle_spectrum(alpha):
    e = [_spectrum_error(alpha, 0.7, M) for M in (8, 16)]
    # the double-layer kernel of the modified Helmholtz operator carries an
    # r^2 log r term, so the smooth rule converges algebraically
    assert e[0] / e[1] > 6, e
    assert e[1] < (2e-7 if alpha == 1.0 else 2e-5), e


def _k0_field(seed, alpha):
    g = np.random.default_rng(seed)
    ang = g.uniform(0, 2 * np.pi, 5)
    rad = g.uniform(1.8, 2.4, 5)
    amp = g.standard_normal(5)
    px, py = rad * np.cos(ang), rad * np.sin(ang)

    def u(x, y):
        r = np.hypot(x[:, None] - px[None, :], y[:, None] - py[None, :])
        return (amp[None, :] * sp.k0(alpha * r)).sum(1)

    def dudn(x, y, nx, ny):
        dx, dy = x[:, None] - px[None, :], y[:, None] - py[None, :]
        r = np.hypot(dx, dy)
        gr = -alpha * sp.k1(alpha * r) / r * amp[None, :]
        return (gr * dx).sum(1) * nx + (gr * dy).sum(1) * ny
    return u, dudn


def _interior_targets(cv, n=24, lim=1.2):
    g1 = np.linspace(-lim, lim, n)
    TX, TY = np.meshgrid(g1, g1)
    tx, ty = TX.ravel(), TY.ravel()
    m = synth.inside_any([cv], tx, ty)
    return tx[m], ty[m]


@pytest.mark.parametrize("kind", ["dirichlet", "neumann"])
@pytest.mark.parametrize("alpha", [1.0, 10.0])
def test_manufactured_k0_sources(kind, alpha):
    cv = synth.Curve(r0=1.0, a=0.3, l1=5)
    tx, ty = _interior_targets(cv)
    nt = len(tx)
    u, dudn = _k0_field(7, alpha)
    errs = []
    for M in (32, 64):
        b = synth.discretize([cv], M)
        ue = np.concatenate([u(tx, ty), u(b["x"], b["y"])])
        if kind == "dirichlet":
            _, uh = bie.solve_dirichlet(alpha, 2e-4, 3, b, None, (tx, ty), np.ones(nt, np.int8), u(b["x"], b["y"]))
        else:
            gN = dudn(b["x"], b["y"], b["nx"], b["ny"])
            _, uh = bie.solve_neumann(alpha, 2e-4, 3, b, None, (tx, ty), np.ones(nt, np.int8), gN)
        e = np.abs(uh - ue) / np.abs(ue).max()
        errs.append((e[:nt].max(), e[nt:].max()))
    errs = np.array(errs)
    assert errs[0, 0] / errs[1, 0] > 5, errs            # panel refinement
    assert errs[1, 0] < 1e-5 and errs[1, 1] < 2e-5, errs


def test_dirichlet_with_volume_source():
    alpha, a, b_ = 1.0, 0.8, -0.5
    cv = synth.Curve(r0=1.0, a=0.3, l1=5)
    tx, ty = _interior_targets(cv, n=12)
    nt = len(tx)
    b = synth.discretize([cv], 48)
    vol = synth.polar_volume(cv, 60, 300)
    ue_f = lambda x, y: np.exp(a * x + b_ * y)
    c = alpha ** 2 - a ** 2 - b_ ** 2
    fv = c * ue_f(vol["x"], vol["y"])
    ft = c * ue_f(np.concatenate([tx, b["x"]]), np.concatenate([ty, b["y"]]))
    gD = ue_f(b["x"], b["y"])
    _, uh = bie.solve_dirichlet(alpha, 4e-4, 3, b, vol, (tx, ty), np.ones(nt, np.int8), gD, fv, ft)
    ue = np.concatenate([ue_f(tx, ty), gD])
    e = np.abs(uh - ue) / np.abs(ue).max()
    assert e[:nt].max() < 5e-6 and e[nt:].max() < 1e-4, (e[:nt].max(), e[nt:].max())


def test_heat_step_closed_form():
    """One implicit-Euler step of the heat equation (elliptic marching,
    Section 1) from u0 = sin(k(x+a)) sin(k(y+b)): (-Lap + alpha^2) u1 =
    alpha^2 u0 has the solution u1 = alpha^2/(alpha^2 + 2k^2) u0, so with that
    boundary data the step must return it at every volume node and boundary
    node, up to the split's local error, which falls with delta."""
    cv = synth.Curve(r0=0.5, a=0.1, l1=3)
    b = synth.discretize([cv], 24)
    k, alpha = np.pi, 3.0
    u0 = lambda x, y: np.sin(k * (x + 0.3)) * np.sin(k * (y + 0.2))
    c = alpha ** 2 / (alpha ** 2 + 2 * k * k)
    errs = []
    for nr, nth, delta in ((24, 96, 2e-3), (32, 128, 1e-3)):
        vol = synth.polar_volume(cv, nr, nth)
        X = np.concatenate([vol["x"], b["x"]])
        Y = np.concatenate([vol["y"], b["y"]])
        _, u1 = bie.heat_step(alpha, delta, 3, b, vol, u0(X, Y), c * u0(b["x"], b["y"]))
        errs.append(np.abs(u1 - c * u0(X, Y)).max() / np.abs(c * u0(X, Y)).max())
    assert errs[0] / errs[1] > 2, errs
    assert errs[1] < 1e-3, errs
