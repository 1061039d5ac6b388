"""CPU FP64 oracle of the boundary integral equation solves (Section 3).

TEST INFRASTRUCTURE ONLY: imported by tests/ (and by the CPU-baseline leg of
bench.py), never by the product package.

* nystrom_matrix: the dense Nystrom matrix of the double-layer operator on the
  boundary nodes, written out from its definition in Section 3.2 (smooth
  panel quadrature; off-diagonal entries w_j alpha/(2 pi) K_1(alpha r)
  (x_i - x_j).nu_j / r with r = |x_i - x_j|, diagonal entries from the
  curvature limit of the double-layer kernel, -w_i kappa_i/(4 pi)).
  K_1 is scipy's modified Bessel function (a library primitive).
* solve_dirichlet / solve_neumann: the discrete systems of Section 3.2,
  (-1/2 I + K) mu = g - V  and  (1/2 I + K) u = V + S[g], solved directly
  (numpy LU, a library primitive), followed by the representations of Section
  2 (u = V[f] + D[mu]; u = V[f] + S[g] - D[u]) evaluated by the split-sum
  oracle at every target.  On the boundary nodes the Dirichlet solution is
  reported as the interior limit V + D[mu] - mu/2 (jump relation of Section
  2) and the Neumann solution as the solved boundary values.
"""
from __future__ import annotations

import numpy as np
from scipy.special import k1

from . import PART_ALL, Problem


def nystrom_rows(boundary, alpha, rows):
    """Rows `rows` of the Nystrom matrix."""
    rows = np.asarray(rows, dtype=np.int64)
    x, y = np.asarray(boundary["x"], float), np.asarray(boundary["y"], float)
    nx, ny = np.asarray(boundary["nx"], float), np.asarray(boundary["ny"], float)
    w, kap = np.asarray(boundary["w"], float), np.asarray(boundary["kappa"], float)
    dx = x[rows, None] - x[None, :]
    dy = y[rows, None] - y[None, :]
    r = np.hypot(dx, dy)
    diag = rows[:, None] == np.arange(len(x))[None, :]
    r[diag] = 1.0
    K = w[None, :] * (alpha / (2.0 * np.pi)) * k1(alpha * r) * (dx * nx[None, :] + dy * ny[None, :]) / r
    K[diag] = (-w * kap / (4.0 * np.pi))[rows]
    return K


def nystrom_matrix(boundary, alpha):
    return nystrom_rows(boundary, alpha, np.arange(len(boundary["x"])))


def _problem(alpha, delta, J, boundary, volume, targets, inside, sigma, mu, f_vol, f_trg):
    nb = len(boundary["x"])
    z = np.zeros(nb)
    return Problem(alpha, delta, J, boundary, volume=volume, targets=targets, inside=inside, on_surface=True,
                   sigma=z if sigma is None else sigma, mu=z if mu is None else mu,
                   f_vol=f_vol, f_trg=f_trg, parts=PART_ALL)


def solve_dirichlet(alpha, delta, J, boundary, volume, targets, inside, g, f_vol=None, f_trg=None):
    """Returns (mu, u): the density on the boundary nodes and u at every
    output (targets, then boundary nodes)."""
    nb = len(boundary["x"])
    nt = len(targets[0])
    if f_vol is not None:
        _, _, V = _problem(alpha, delta, J, boundary, volume, targets, inside, None, None, f_vol, f_trg).eval()
    else:
        V = np.zeros(nt + nb)
    A = -0.5 * np.eye(nb) + nystrom_matrix(boundary, alpha)
    mu = np.linalg.solve(A, np.asarray(g, float) - V[nt:])
    _, D, _ = _problem(alpha, delta, J, boundary, volume, targets, inside, None, mu, None, None).eval()
    u = V + D
    u[nt:] -= 0.5 * mu
    return mu, u


def solve_neumann(alpha, delta, J, boundary, volume, targets, inside, g, f_vol=None, f_trg=None):
    """Returns (ub, u): the solution on the boundary nodes and u at every
    output (targets, then boundary nodes)."""
    nb = len(boundary["x"])
    nt = len(targets[0])
    S, _, V = _problem(alpha, delta, J, boundary, volume, targets, inside, g, None, f_vol, f_trg).eval()
    if f_vol is None:
        V = np.zeros(nt + nb)
    A = 0.5 * np.eye(nb) + nystrom_matrix(boundary, alpha)
    ub = np.linalg.solve(A, V[nt:] + S[nt:])
    _, D, _ = _problem(alpha, delta, J, boundary, volume, targets, inside, None, ub, None, None).eval()
    u = V + S - D
    u[nt:] = ub
    return ub, u


def heat_step(alpha, delta, J, boundary, volume, u_n, g_next, F=None):
    """One implicit-Euler step of u_t = Lap u + F with time step 1/alpha^2
    (elliptic marching, Section 1): (-Lap + alpha^2) u^{n+1} = alpha^2 u^n +
    F^{n+1} with u^{n+1} = g_next on the boundary, solved as the Dirichlet
    problem above with the volume nodes as targets.  u_n and F are given at
    the outputs (volume nodes, then boundary nodes); returns (mu, u^{n+1})."""
    f = alpha ** 2 * np.asarray(u_n, float) + (0.0 if F is None else np.asarray(F, float))
    nv = len(volume["x"])
    targets = (volume["x"], volume["y"])
    inside = np.ones(nv, np.int8)
    return solve_dirichlet(alpha, delta, J, boundary, volume, targets, inside, g_next, f[:nv], f)
