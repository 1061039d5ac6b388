"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: Bessel
closed forms, scipy quadrature of the defining time integrals, the circle
and disk closed forms, Green's representation formula, and the convergence
orders the paper states for the local expansions (Section 4.1: first order
kept, error O(delta*^{3/2})).  A dropped term, a wrong sign or index in the
oracle fails at least one of them.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp
from scipy import integrate

import oracle as O
import synth


# --------------------------------------------------------------------------
# (a) kernel split, Section 2.1: G^R(delta*) + sum_j K_j + G^H(delta) = K0/2pi
# --------------------------------------------------------------------------
@pytest.mark.parametrize("alpha,delta,J", [(10.0, 0.04, 3), (1.0, 2e-5, 3), (100.0, 1e-4, 2), (3.0, 1e-3, 0)])
def test_split_sums_to_green(alpha, delta, J):
    ds = delta / 4 ** J
    for r in np.geomspace(1e-4, 3.0, 23):
        if sp.k0(alpha * r) < 1e-280:
            continue
        tot = O.GR(r, alpha, ds) + sum(O.KS(r, alpha, delta, j) for j in range(1, J + 1)) + O.GH(r, alpha, delta)
        ex = sp.k0(alpha * r) / (2 * np.pi)
        assert abs(tot - ex) <= 2e-14 * ex, (r, tot, ex)


@pytest.mark.parametrize("alpha,delta,J", [(10.0, 0.04, 3), (1.0, 2e-5, 3), (100.0, 1e-4, 2)])
def test_split_sums_to_double_layer_kernel(alpha, delta, J):
    """nu'.(x-x') * [G^R_D + sum_j K_j^D + G^H_D] is the double-layer kernel
    alpha K1(alpha r) nu'.(x-x')/(2 pi r) of Section 3.3; G^R_D is the
    t in [0, delta*] integral of H/(2t), here by scipy."""
    ds = delta / 4 ** J
    for r in np.geomspace(3e-4, 2.0, 17):
        if sp.k1(alpha * r) < 1e-280:
            continue
        a = r * r / (4 * ds)
        grd = integrate.quad(lambda u: math.exp(-a * math.exp(u) - alpha ** 2 * ds * math.exp(-u) + u),
                             0, max(1.0, math.log(800 / a)), limit=400, epsabs=0, epsrel=1e-13)[0] / (8 * math.pi * ds)
        tot = grd + sum(O.KD(r, alpha, delta, j) for j in range(1, J + 1)) + O.GHD(r, alpha, delta)
        ex = alpha * sp.k1(alpha * r) / (2 * np.pi * r)
        assert abs(tot - ex) <= 1e-13 * ex, (r, tot, ex)


def test_special_values():
    alpha, delta = 10.0, 0.01
    # G^H(0) = E1(alpha^2 delta)/4pi, K_j^S(0) = [E1(a^2 d/4^j) - E1(a^2 d/4^(j-1))]/4pi
    assert O.GH(0.0, alpha, delta) == pytest.approx(sp.exp1(alpha ** 2 * delta) / (4 * np.pi), rel=1e-14)
    for j in (1, 2, 3):
        ex = (sp.exp1(alpha ** 2 * delta / 4 ** j) - sp.exp1(alpha ** 2 * delta / 4 ** (j - 1))) / (4 * np.pi)
        assert O.KS(0.0, alpha, delta, j) == pytest.approx(ex, rel=1e-13)
    # history kernel = K0/2pi - G^R, both routes
    assert O.GH(0.07, alpha, delta) == pytest.approx(sp.k0(0.7) / (2 * np.pi) - O.GR(0.07, alpha, delta), rel=1e-13)


def test_incomplete_bessel_convention():
    """Eq. (diffker_dlp) with K_nu(x,y) = int_1^inf s^(nu-1) exp(-xs-y/s) ds
    equals the time integral of H/(2t) over level j (the other index
    convention differs by an order of magnitude)."""
    alpha, delta, r = 10.0, 0.04, 0.07

    def Kinc(nu, x, y):
        return integrate.quad(lambda s: s ** (nu - 1) * math.exp(-x * s - y / s), 1, np.inf,
                              epsabs=0, epsrel=1e-13, limit=200)[0]
    for j in (1, 2, 3):
        paper = (4 ** (j - 2) / (2 * np.pi * delta)) * Kinc(1, 4 ** (j - 2) * r * r / delta, alpha ** 2 * delta / 4 ** (j - 1)) \
            - (4 ** (j - 1) / (2 * np.pi * delta)) * Kinc(1, 4 ** (j - 1) * r * r / delta, alpha ** 2 * delta / 4 ** j)
        assert O.KD(r, alpha, delta, j) == pytest.approx(paper, rel=1e-11)
        paperS = (Kinc(0, 4 ** (j - 2) * r * r / delta, alpha ** 2 * delta / 4 ** (j - 1))
                  - Kinc(0, 4 ** (j - 1) * r * r / delta, alpha ** 2 * delta / 4 ** j)) / (4 * np.pi)
        assert O.KS(r, alpha, delta, j) == pytest.approx(paperS, rel=1e-11)
    assert O.KD(0.07, 10.0, 0.04, 2) == pytest.approx(5.5612488764522, rel=1e-12)


@pytest.mark.parametrize("alpha,delta", [(10.0, 1e-3), (3.0, 4e-3)])
def test_history_kernel_is_fourier_multiplier(alpha, delta):
    """G^H is the radial inverse transform of the history multiplier of
    eq. (sh): (1/2pi) int_0^inf exp(-delta(a^2+k^2))/(a^2+k^2) J0(kr) k dk."""
    kc = math.sqrt(60 / delta)
    for r in (0.0, 0.01, 0.05, 0.2):
        f = lambda k: math.exp(-delta * (alpha ** 2 + k * k)) / (alpha ** 2 + k * k) * sp.j0(k * r) * k
        v = integrate.quad(f, 0, kc, limit=4000, epsabs=0, epsrel=1e-13)[0] / (2 * np.pi)
        assert O.GH(r, alpha, delta) == pytest.approx(v, rel=1e-11)


# --------------------------------------------------------------------------
# Local expansions, Section 4.1
# --------------------------------------------------------------------------
def test_local_coefficients_small_c2_limits():
    """Remark 4.2 (P_m, Q_m), the U_m remark and Remark 4.9 (W_0, W_1) at
    c2 -> 0, and the c1 = 0 values behind Corollaries 4.4, 4.7 and 4.10."""
    for c1 in (0.0, 0.3, 1.0, 2.5, 6.0):
        E = sp.erfc(c1 / 2)
        G = 2 / math.sqrt(math.pi) * math.exp(-c1 * c1 / 4)
        c = O.local_coeffs(c1, 1e-4)
        for m in range(4):
            assert c[f"P{m}"] == pytest.approx(2 * c1 ** m * (G - c1 * E), abs=1e-7)
        for m in range(2):
            assert c[f"Q{m}"] == pytest.approx(2 / 3 * c1 ** m * ((2 - c1 ** 2) * G + c1 ** 3 * E), abs=1e-7)
        for m in range(5):
            assert c[f"U{m}"] == pytest.approx(2 * c1 ** m * E, abs=1e-7)
        assert c["W0"] == pytest.approx(4 - (2 + c1 ** 2) * E + c1 * G, abs=1e-7)
        assert c["W1"] == pytest.approx(4 - 2 * E + c1 * G / 3 + (c1 ** 4 * E - c1 ** 3 * G) / 6, abs=1e-6)
    for c2 in (1e-3, 0.1, 0.7, 2.0):
        c = O.local_coeffs(0.0, c2)
        # Cor. 4.4: sqrt(d*) P0/4 = sqrt(d*) erf(c2)/(2 c2)
        assert c["P0"] / 4 == pytest.approx(sp.erf(c2) / (2 * c2), rel=1e-13)
        # Cor. 4.4, d*^{3/2} kappa^2/32 (Q0 + 3 P2): P2 = 0 at c1 = 0
        with mpmath.workdps(40):
            q0 = (2 * mpmath.erf(c2) - 4 * c2 / mpmath.sqrt(mpmath.pi) * mpmath.exp(-c2 * c2)) / mpmath.mpf(c2) ** 3
        assert c["Q0"] == pytest.approx(float(q0), rel=1e-13)
        # Cor. 4.10: d f W0/4 = d f (1 - exp(-c2^2))/(2 c2^2)
        assert c["W0"] / 4 == pytest.approx(-math.expm1(-c2 * c2) / (2 * c2 * c2), rel=1e-13)
        assert c["U0"] == pytest.approx(2.0, rel=1e-15)


def _gr_scipy(r, alpha, d):
    """int_0^d H(t, r) dt by scipy (u = r^2/4t substitution)."""
    if r == 0:
        return np.inf
    a = r * r / (4 * d)
    return integrate.quad(lambda s: math.exp(-s - alpha ** 2 * r * r / (4 * s)) / s, a, np.inf,
                          epsabs=0, epsrel=1e-12, limit=200)[0] / (4 * math.pi)


def test_local_layer_vs_brute_force_circle():
    """S_{L,A} and D_{L,A} (t in [0, delta*]) on a circle with an oscillating
    density, by adaptive quadrature of the time-integrated kernel over the
    arc; the oracle's local part (Lemmas 4.1, 4.5, first order) converges at
    O(delta*^{3/2}) or faster, inside and outside."""
    R, alpha, n = 0.5, 10.0, 3
    bnd = synth.discretize([synth.Curve(r0=R)], 48)
    sig = np.cos(n * bnd["t"]) + 0.3
    errs = {}
    for ds in (4e-4, 1e-4, 2.5e-5):
        sq = math.sqrt(ds)
        pts = [(R - 1.5 * sq, 0.3, 1), (R + 2.0 * sq, 1.1, 0), (R - 0.4 * sq, 2.0, 1)]
        tx = np.array([p[0] * math.cos(p[1]) for p in pts])
        ty = np.array([p[0] * math.sin(p[1]) for p in pts])
        ins = np.array([p[2] for p in pts])
        P = O.Problem(alpha, ds, 0, bnd, targets=(tx, ty), inside=ins, sigma=sig, mu=sig, parts=O.PART_LOCAL)
        S, D, _ = P.eval()
        for k, (rr, th, _) in enumerate(pts):
            x = np.array([rr * math.cos(th), rr * math.sin(th)])

            def dist(tp):
                return math.hypot(x[0] - R * math.cos(tp), x[1] - R * math.sin(tp))

            def fs(tp):
                return _gr_scipy(dist(tp), alpha, ds) * (math.cos(n * tp) + 0.3) * R

            def fd(tp):
                r = dist(tp)
                a = r * r / (4 * ds)
                grd = integrate.quad(lambda u: math.exp(-a * math.exp(u) - alpha ** 2 * ds * math.exp(-u) + u),
                                     0, max(1.0, math.log(800 / a)), epsabs=0, epsrel=1e-12, limit=200)[0] / (8 * math.pi * ds)
                nd = (x[0] - R * math.cos(tp)) * math.cos(tp) + (x[1] - R * math.sin(tp)) * math.sin(tp)
                return grd * nd * (math.cos(n * tp) + 0.3) * R
            w = 14 * sq / R
            brk = [th - w, th - w / 4, th, th + w / 4, th + w]
            s_ref = sum(integrate.quad(fs, brk[i], brk[i + 1], epsabs=1e-15, epsrel=1e-11, limit=200)[0] for i in range(4))
            d_ref = sum(integrate.quad(fd, brk[i], brk[i + 1], epsabs=1e-15, epsrel=1e-11, limit=200)[0] for i in range(4))
            errs.setdefault(k, []).append((abs(S[k] - s_ref), abs(D[k] - d_ref)))
    for k, e in errs.items():
        e = np.array(e)
        # S error O(ds^{3/2}) => ratio >= ~8 per factor 4; D likewise
        assert e[0, 0] / e[2, 0] > 40, (k, e)
        assert e[0, 1] / e[2, 1] > 40, (k, e)
        assert e[2, 0] < 2e-6 and e[2, 1] < 1e-5, (k, e)


def test_local_volume_vs_brute_force_disk():
    """V_L = int_0^delta int_disk H dt dx' for f = 1 near the boundary of a
    disk (Lemma 4.8 first order: delta W0/4, error O(delta^{3/2})), and the
    far-field corollary 4.11 at the centre."""
    R, alpha = 0.5, 10.0
    bnd = synth.discretize([synth.Curve(r0=R)], 32)

    def mass(t, rho):  # Gaussian of variance 2t centred at distance rho: mass in disk
        f = lambda s: s / (2 * t) * math.exp(-(s - rho) ** 2 / (4 * t)) * sp.ive(0, s * rho / (2 * t))
        lo, hi = max(0.0, rho - 40 * math.sqrt(t)), min(R, rho + 40 * math.sqrt(t))
        return integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-12, limit=200)[0] if hi > lo else 0.0

    errs, nxt = [], []
    for d in (1e-3, 2.5e-4, 6.25e-5):
        rho = R - 1.2 * math.sqrt(d)
        ref = integrate.quad(lambda t: math.exp(-alpha ** 2 * t) * mass(t, rho), 0, d, epsabs=0, epsrel=1e-11, limit=200)[0]
        P = O.Problem(alpha, d, 0, bnd, targets=(np.array([rho]), np.array([0.0])), inside=np.array([1]),
                      f_trg=np.array([1.0]), parts=O.PART_LOCAL)
        _, _, V = P.eval()
        errs.append(abs(V[0] - ref))
        # the first neglected term of Lemma 4.8, delta^{3/2}(2 f_eta - f kappa0) Q0/8
        # with f = 1, kappa0 = 1/R, accounts for the error to the next order
        q0 = O.local_coeffs(1.2, alpha * math.sqrt(d))["Q0"]
        nxt.append(abs(V[0] - d ** 1.5 * (1 / R) * q0 / 8 - ref))
        # far from the boundary: Cor. 4.11 with f = 1 is exact (no curvature)
        P = O.Problem(alpha, d, 0, bnd, targets=(np.array([0.0]), np.array([0.0])), inside=np.array([1]),
                      f_trg=np.array([1.0]), parts=O.PART_LOCAL)
        _, _, V0 = P.eval()
        assert V0[0] == pytest.approx(-math.expm1(-alpha ** 2 * d) / alpha ** 2, rel=1e-14)
    assert errs[0] / errs[2] > 30, errs
    assert errs[2] < 3e-7, errs
    assert all(n < 0.1 * e for n, e in zip(nxt, errs)), (nxt, errs)


# --------------------------------------------------------------------------
# (d) full potentials: circle and disk closed forms
# --------------------------------------------------------------------------
def test_circle_closed_forms_full_split():
    """S[cos n th] = R I_n(a r) K_n(a R) cos n th and D = R a I_n K_n'(a R)
    cos n th inside a circle; all three parts of the split summed, error
    O(delta*^{3/2}) near the boundary, exact (to quadrature) far away."""
    R, alpha, n = 0.5, 10.0, 3
    b = synth.discretize([synth.Curve(r0=R)], 32)
    sig = np.cos(n * b["t"])
    pts = [(0.3, 0.2), (R - 0.02, 0.1), (R - 0.004, 0.7), (R - 0.0015, 1.3)]
    tx = np.array([p[0] * np.cos(p[1]) for p in pts]); ty = np.array([p[0] * np.sin(p[1]) for p in pts])
    Sex = np.array([R * sp.iv(n, alpha * p[0]) * sp.kv(n, alpha * R) * np.cos(n * p[1]) for p in pts])
    Dex = np.array([R * alpha * sp.iv(n, alpha * p[0]) * sp.kvp(n, alpha * R) * np.cos(n * p[1]) for p in pts])
    e = []
    for delta in (4e-3, 1e-3, 2.5e-4):
        P = O.Problem(alpha, delta, 3, b, targets=(tx, ty), inside=np.ones(len(tx)), sigma=sig, mu=sig)
        S, D, _ = P.eval()
        assert abs(S[0] - Sex[0]) < 1e-15 and abs(D[0] - Dex[0]) < 1e-15
        e.append((np.abs(S - Sex)[2:].max(), np.abs(D - Dex)[2:].max()))
    e = np.array(e)
    assert np.all(e[0] / e[2] > 40), e
    assert e[2, 0] < 5e-8 and e[2, 1] < 2e-7, e


def test_local_volume_exterior_disk():
    """Exterior targets near a disk (the complement-domain reading of Lemma
    4.8): V_L = int_0^delta int_disk H dt dx' for f = 1 against the first-
    order formula delta f0 [(1 - e^{-c2^2})/c2^2 - W0/4], converging at order
    3/2; the next term of Lemma 4.8 for the complement (curvature -kappa)
    accounts for the error."""
    R, alpha = 0.5, 10.0
    bnd = synth.discretize([synth.Curve(r0=R)], 32)
    nb = len(bnd["x"])

    def mass(t, rho):
        f = lambda s: s / (2 * t) * math.exp(-(s - rho) ** 2 / (4 * t)) * sp.ive(0, s * rho / (2 * t))
        lo, hi = max(0.0, rho - 40 * math.sqrt(t)), min(R, rho + 40 * math.sqrt(t))
        return integrate.quad(f, lo, hi, epsabs=0, epsrel=1e-12, limit=200)[0] if hi > lo else 0.0

    errs, nxt = [], []
    for d in (1e-3, 2.5e-4, 6.25e-5):
        rho = R + 1.2 * math.sqrt(d)
        ref = integrate.quad(lambda t: math.exp(-alpha ** 2 * t) * mass(t, rho), 0, d, epsabs=0, epsrel=1e-11,
                             limit=200)[0]
        # f on the boundary nodes comes from the on-surface entries of f_trg;
        # the exterior target's own entry is not used
        P = O.Problem(alpha, d, 0, bnd, targets=(np.array([rho]), np.array([0.0])), inside=np.array([0]),
                      on_surface=True, f_trg=np.concatenate([[7.0], np.ones(nb)]), parts=O.PART_LOCAL)
        _, _, V = P.eval()
        errs.append(abs(V[0] - ref))
        q0 = O.local_coeffs(1.2, alpha * math.sqrt(d))["Q0"]
        nxt.append(abs(V[0] - d ** 1.5 * (1 / R) * q0 / 8 - ref))
    assert errs[0] / errs[2] > 30, errs
    assert errs[2] < 2e-7, errs
    assert all(n < e / 10 for n, e in zip(nxt, errs)), (nxt, errs)
    # without f on the boundary the exterior local part is unknown: NaN
    P = O.Problem(alpha, 1e-3, 0, bnd, targets=(np.array([R + 0.01]), np.array([0.0])), inside=np.array([0]),
                  f_trg=np.array([1.0]), parts=O.PART_LOCAL)
    assert np.isnan(P.eval()[2][0])


def test_disk_volume_exterior_closed_form():
    """V[1] outside a disk, (R/a) I1(a R) K0(a r): history + exterior local
    part (polar volume rule) within the band converging at order 3/2 in
    delta, and exact beyond the band (history part alone)."""
    R, alpha = 0.5, 10.0
    cv = synth.Curve(r0=R)
    b = synth.discretize([cv], 16)
    nb = len(b["x"])
    vol = synth.polar_volume(cv, 80, 400)
    rr = R + np.array([0.001, 0.01, 0.3])
    ex = R * sp.i1(alpha * R) * sp.k0(alpha * rr) / alpha
    e = []
    for d in (8e-4, 5e-5):
        P = O.Problem(alpha, d, 3, b, volume=vol, targets=(rr, np.zeros(3)), inside=np.zeros(3), on_surface=True,
                      f_vol=np.ones(len(vol["x"])), f_trg=np.ones(3 + nb), parts=O.PART_HISTORY | O.PART_LOCAL)
        _, _, V = P.eval()
        e.append(np.abs(V[:3] - ex) / np.abs(ex).max())
    e = np.array(e)
    assert np.all(e[0, :2] / e[1, :2] > 30), e           # 16x delta: order 3/2 gives 64
    assert e[1, :2].max() < 5e-5 and e[1, 2] < 1e-14, e


def test_disk_volume_closed_form():
    """V[1] inside a disk: (1 - a R K1(a R) I0(a r))/a^2 (history + local,
    polar volume rule), at targets farther than sqrt(delta)(12 + 2 a sqrt(delta))
    from the circle where the local part with f = 1 is exact (Cor. 4.11)."""
    R, alpha = 0.5, 10.0
    cv = synth.Curve(r0=R)
    b = synth.discretize([cv], 16)
    vol = synth.polar_volume(cv, 80, 400)
    rr = np.array([0.0, 0.2, 0.3])
    ex = (1 - alpha * R * sp.k1(alpha * R) * sp.i0(alpha * rr)) / alpha ** 2
    P = O.Problem(alpha, 2e-4, 3, b, volume=vol, targets=(rr, np.zeros(3)), inside=np.ones(3),
                  f_vol=np.ones(len(vol["x"])), f_trg=np.ones(3), parts=O.PART_HISTORY | O.PART_LOCAL)
    _, _, V = P.eval()
    assert np.allclose(V, ex, rtol=0, atol=1e-9 * abs(ex).max()), (V, ex)


def test_volume_history_of_gaussian():
    """V_H of f = exp(-|x-c|^2/s^2): the history part of the free-space volume
    potential is (s^2/2) int exp(-k^2 s^2/4 - delta(a^2+k^2)) J0(kr) k/(a^2+k^2) dk."""
    alpha, s, delta = 10.0, 0.1, 1e-3
    cv = synth.Curve(r0=1.0, a=0.3, l1=5)
    b = synth.discretize([cv], 16)
    vol = synth.polar_volume(cv, 60, 300)
    c = (0.1, -0.05)
    f = np.exp(-((vol["x"] - c[0]) ** 2 + (vol["y"] - c[1]) ** 2) / s ** 2)
    tx = np.array([0.1, 0.15, 0.0, 0.3]); ty = np.array([-0.05, 0.0, 0.2, -0.1])
    P = O.Problem(alpha, delta, 3, b, volume=vol, targets=(tx, ty), inside=np.ones(4), f_vol=f,
                  parts=O.PART_HISTORY)
    _, _, V = P.eval()
    for k in range(4):
        r = math.hypot(tx[k] - c[0], ty[k] - c[1])
        g = lambda q: math.exp(-q * q * s * s / 4 - delta * (alpha ** 2 + q * q)) * sp.j0(q * r) * q / (alpha ** 2 + q * q)
        ref = 0.5 * s * s * integrate.quad(g, 0, 300, limit=2000, epsabs=0, epsrel=1e-13)[0]
        assert V[k] == pytest.approx(ref, rel=1e-10)


def _graded_polar_rule(cx, cy, rad, h0, n_theta=96, nq=20):
    """Area rule on the disk of radius rad about (cx, cy): Gauss-Legendre in
    the radius on panels [0, h0], [h0, 2 h0], [2 h0, 4 h0], ... (graded
    towards the centre, where the history kernel peaks over a width
    sqrt(delta)), trapezoidal in the angle.  Test quadrature only."""
    tg, wg = np.polynomial.legendre.leggauss(nq)
    edges = [0.0, h0]
    while edges[-1] < rad:
        edges.append(min(rad, 2 * edges[-1]))
    rho, wr = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        rho.append(0.5 * (a + b) + 0.5 * (b - a) * tg)
        wr.append(0.5 * (b - a) * wg)
    rho, wr = np.concatenate(rho), np.concatenate(wr)
    th = (np.arange(n_theta) + 0.5) * (2 * np.pi / n_theta)
    X = cx + rho[:, None] * np.cos(th)[None, :]
    Y = cy + rho[:, None] * np.sin(th)[None, :]
    W = (wr * rho)[:, None] * np.full(n_theta, 2 * np.pi / n_theta)[None, :]
    return {"x": X.ravel(), "y": Y.ravel(), "w": W.ravel()}


@pytest.mark.parametrize("d", [0.0, 0.05, 0.12])
def test_volume_potential_of_gaussian_full_split(d):
    """Spec invariant (c): the whole V = V_H + V_L of the Gaussian
    source f = exp(-|x-c|^2/s^2) against the free-space closed form
    (s^2/2) int_0^inf exp(-k^2 s^2/4) J0(k d) k/(alpha^2 + k^2) dk (Section
    2.1, eq. (vp); at d = 0 it is (s^2/4) e^{a^2 s^2/4} E1(a^2 s^2/4)).  The
    target lies farther from the boundary than sqrt(delta)(12 + 2 alpha
    sqrt(delta)), so the oracle's local part is Corollary 4.11 at first
    order: delta f(x)(1 - e^{-alpha^2 delta})/(alpha^2 delta).  The exact
    local integral is int_0^delta e^{-alpha^2 t} (e^{t Lap} f)(x) dt =
    delta f + delta^2/2 (Lap f - alpha^2 f) + O(delta^3), and the first-order
    term expands to delta f - alpha^2 delta^2 f/2, so the oracle's error must
    be -delta^2/2 (Lap f)(x) + O(delta^3): a dropped or mis-signed local term
    leaves an O(delta) error instead."""
    alpha, s = 10.0, 0.1
    tx, ty = 0.05, -0.02                         # the target; the Gaussian sits at distance d
    c = (tx - d, ty)
    if d == 0.0:
        ex = s * s / 4 * math.exp(alpha ** 2 * s ** 2 / 4) * sp.exp1(alpha ** 2 * s ** 2 / 4)
        assert ex == pytest.approx(0.003352213612078, rel=1e-12)
    else:
        g = lambda q: math.exp(-q * q * s * s / 4) * sp.j0(q * d) * q / (alpha ** 2 + q * q)
        ex = 0.5 * s * s * integrate.quad(g, 0, 400, limit=4000, epsabs=0, epsrel=1e-13)[0]
    lap = (4 * d * d / s ** 4 - 4 / s ** 2) * math.exp(-d * d / s ** 2)
    rad = 0.7                                     # f < 1e-16 beyond: the disk is free space
    b = synth.discretize([synth.Curve(r0=rad, cx=tx, cy=ty)], 16)
    errs, errs2 = [], []
    for delta, rtol in ((1e-4, 0.07), (2.5e-5, 0.02)):
        vol = _graded_polar_rule(tx, ty, rad, 0.25 * math.sqrt(delta))
        f = np.exp(-((vol["x"] - c[0]) ** 2 + (vol["y"] - c[1]) ** 2) / s ** 2)
        fx = math.exp(-d * d / s ** 2)
        P = O.Problem(alpha, delta, 3, b, volume=vol, targets=(np.array([tx]), np.array([ty])),
                      inside=np.ones(1), f_vol=f, f_trg=np.array([fx]))
        _, _, V = P.eval()
        err = V[0] - ex
        errs.append(err)
        assert err == pytest.approx(-0.5 * delta ** 2 * lap, rel=rtol), (delta, err, -0.5 * delta ** 2 * lap)
        # second order (Corollary 4.11 with f_xx + f_yy): the O(delta^2) error
        # is removed and what is left is O(delta^3)
        gx, gy = -2 * (tx - c[0]) / s ** 2 * fx, -2 * (ty - c[1]) / s ** 2 * fx
        hxx = (4 * (tx - c[0]) ** 2 / s ** 4 - 2 / s ** 2) * fx
        hyy = (4 * (ty - c[1]) ** 2 / s ** 4 - 2 / s ** 2) * fx
        hxy = 4 * (tx - c[0]) * (ty - c[1]) / s ** 4 * fx
        assert hxx + hyy == pytest.approx(lap, rel=1e-12)
        fj = np.array([[gx], [gy], [hxx], [hxy], [hyy]])
        P2 = O.Problem(alpha, delta, 3, b, volume=vol, targets=(np.array([tx]), np.array([ty])),
                       inside=np.ones(1), f_vol=f, f_trg=np.array([fx]), f_jet=fj, local_order=2)
        errs2.append(P2.eval()[2][0] - ex)
    assert errs[0] / errs[1] == pytest.approx(16.0, rel=0.1), errs
    assert abs(errs2[1]) < 0.02 * abs(errs[1]) and abs(errs2[0] / errs2[1]) > 40, (errs, errs2)


# --------------------------------------------------------------------------
# (b) Green's representation formula, eq. (sol_neumann) with f = 0
# --------------------------------------------------------------------------
def test_green_representation_starfish():
    """u = S[du/dn] - D[u] inside, u/2 on the boundary, for u a sum of K0
    sources outside the config-0 starfish (Section 6.1 setup); error
    O(delta*^{3/2})."""
    alpha = 10.0
    cv = synth.Curve(r0=1.0, a=0.3, l1=5)
    b = synth.discretize([cv], 64)
    tp = np.linspace(0, 2 * np.pi, 10, endpoint=False) + 0.1
    g, g1, _ = cv.eval(tp)
    p = g + 0.2 * (g1.imag - 1j * g1.real) / np.abs(g1)

    def u(x, y):
        return sum(10.0 * sp.k0(alpha * np.abs(x + 1j * y - pj)) for pj in p)

    def dudn(x, y, nx, ny):
        out = 0
        for pj in p:
            d = x + 1j * y - pj; r = np.abs(d)
            out = out - 10.0 * alpha * sp.k1(alpha * r) * (d.real * nx + d.imag * ny) / r
        return out
    sig = dudn(b["x"], b["y"], b["nx"], b["ny"]); mu = u(b["x"], b["y"])
    t0 = np.array([0.3, 1.1, 2.5, 4.0])
    g0, g10, _ = cv.eval(t0); n0 = (g10.imag - 1j * g10.real) / np.abs(g10)
    z = np.concatenate([[0.1 + 0.2j, -0.3 + 0.1j]] + [g0 - h * n0 for h in (0.05, 0.01, 0.003, 0.001)])
    tx, ty = z.real, z.imag
    e = []
    for delta in (4e-3, 2.5e-4):
        P = O.Problem(alpha, delta, 3, b, targets=(tx, ty), inside=np.ones(len(tx)), on_surface=True,
                      sigma=sig, mu=mu)
        S, D, _ = P.eval()
        err = S - D - np.concatenate([u(tx, ty), 0.5 * mu])
        e.append((np.abs(err[:len(tx)]).max(), np.abs(err[len(tx):]).max()))
    e = np.array(e)
    assert np.all(e[0] / e[1] > 30), e            # 4^3 ratio in delta => >= 64^{1/2}... order 3/2 gives 64
    assert e[1, 0] < 4e-6 and e[1, 1] < 3e-5, e


# --------------------------------------------------------------------------
# Geometry helpers of the oracle: refinement and closest point
# --------------------------------------------------------------------------
def test_refined_levels_on_curve():
    cv = synth.Curve(r0=1.0, a=0.3, l1=5)
    b = synth.discretize([cv], 64)
    sig = np.cos(3 * b["t"])
    P = O.Problem(10.0, 1e-3, 3, b, sigma=sig, mu=sig)
    per = cv.perimeter(1 << 16)
    tg, _ = synth.gauss_legendre()
    for j in (1, 2, 3):
        L = P.refine(j)
        assert L["w"].sum() == pytest.approx(per, rel=1e-12)
        # child node k of child c of panel p sits at the child's GL node in t
        M, nch = 64, 1 << j
        edges = np.linspace(0, 2 * np.pi, M + 1)
        h = (edges[1] - edges[0]) / nch
        t = (edges[:-1, None, None] + h * (np.arange(nch)[None, :, None] + 0.5 * (1 + tg[None, None, :]))).ravel()
        gx, _, _ = cv.eval(t)
        assert np.abs(L["x"] + 1j * L["y"] - gx).max() < 1e-12
        assert np.abs(L["sigma"] - np.cos(3 * t)).max() < 1e-10


def test_closest_point_brute_force():
    cv = synth.Curve(r0=1.0, a=0.3, l1=5)
    b = synth.discretize([cv], 64)
    P = O.Problem(10.0, 1e-3, 3, b)
    g = np.random.default_rng(7)
    tt = np.linspace(0, 2 * np.pi, 400001)
    gx, _, _ = cv.eval(tt)
    for _ in range(20):
        t0 = g.uniform(0, 2 * np.pi)
        z0, z1, _ = cv.eval(np.array([t0]))
        n = (z1.imag - 1j * z1.real) / np.abs(z1)
        p = (z0 + g.uniform(-0.05, 0.05) * n)[0]
        cp = P.closest(p.real, p.imag)
        dmin = np.abs(gx - p).min()
        assert cp["r"] <= dmin + 1e-10
        assert cp["r"] >= dmin - 1e-7


# --------------------------------------------------------------------------
# Second-order local expansions (local_order = 2): the printed delta*^{3/2}
# and delta*^2 terms of Lemmas 4.1, 4.5, 4.8 and Corollaries 4.4, 4.7, 4.10,
# 4.11.  With them the local error falls from O(delta*^{3/2}) to
# O(delta*^{5/2}) (O(delta^3) far from the boundary): a factor of 16 in
# delta* divides it by ~1000 instead of ~64.
# --------------------------------------------------------------------------
def _layer_brute(cv, x, t0, ds, alpha, dens):
    """S_{L,A} and D_{L,A} at x by adaptive quadrature over the curve
    parameter near t0 of the time-integrated kernel (the density dens(t) in
    the curve parameter)."""
    sq = math.sqrt(ds)

    def geo(tp):
        g, g1, _ = cv.eval(np.array([tp]))
        return g[0], g1[0]

    def fs(tp):
        g, g1 = geo(tp)
        return _gr_scipy(abs(complex(*x) - g), alpha, ds) * dens(tp) * abs(g1)

    def fd(tp):
        g, g1 = geo(tp)
        r = abs(complex(*x) - g)
        a = r * r / (4 * ds)
        grd = integrate.quad(lambda u: math.exp(-a * math.exp(u) - alpha ** 2 * ds * math.exp(-u) + u),
                             0, max(1.0, math.log(800 / max(a, 1e-300))), epsabs=0, epsrel=1e-12,
                             limit=200)[0] / (8 * math.pi * ds)
        nu = (g1.imag - 1j * g1.real) / abs(g1)
        dd = complex(*x) - g
        return grd * (dd.real * nu.real + dd.imag * nu.imag) * dens(tp) * abs(g1)
    w = 14 * sq / 0.45
    brk = [t0 - w, t0 - w / 4, t0, t0 + w / 4, t0 + w]
    s = sum(integrate.quad(fs, brk[i], brk[i + 1], epsabs=1e-16, epsrel=1e-12, limit=300)[0] for i in range(4))
    d = sum(integrate.quad(fd, brk[i], brk[i + 1], epsabs=1e-16, epsrel=1e-12, limit=300)[0] for i in range(4))
    return s, d


@pytest.mark.parametrize("curve", ["circle", "star3"])
def test_local_layer_order2_vs_brute_force(curve):
    """S_{L,A}, D_{L,A} with the second-order terms (Lemmas 4.1, 4.5;
    Corollaries 4.4, 4.7) against brute-force quadrature, with the oscillating
    density cos 3t + 0.3, off the curve on both sides and at a boundary node.
    The 3-armed curve has non-constant curvature (gamma''' != 0).  Reading:
    the gamma'''' term of Lemma 4.5's delta*^{3/2} bracket multiplies
    (3 Q0 + P2); with the printed grouping under (3 Q0 - U3) the D error
    stays O(delta*^{3/2})."""
    alpha = 10.0
    cv = synth.Curve(r0=0.5) if curve == "circle" else synth.Curve(r0=0.5, a=0.06, l1=3)
    bnd = synth.discretize([cv], 48 if curve == "circle" else 64)
    sig = np.cos(3 * bnd["t"]) + 0.3
    dens = lambda t: math.cos(3 * t) + 0.3
    node = 37                                     # an on-surface target
    errs = []
    for ds in (4e-4, 2.5e-5):
        sq = math.sqrt(ds)
        specs = [(0.3, -1.5 * sq), (1.1, 2.0 * sq), (2.0, -0.4 * sq)]
        tx, ty, ins = [], [], []
        for t0, off in specs:
            g, g1, _ = cv.eval(np.array([t0]))
            z = g[0] + off * (g1[0].imag - 1j * g1[0].real) / abs(g1[0])
            tx.append(z.real); ty.append(z.imag); ins.append(1 if off < 0 else 0)
        P = O.Problem(alpha, ds, 0, bnd, targets=(np.array(tx), np.array(ty)), inside=np.array(ins),
                      on_surface=True, sigma=sig, mu=sig, parts=O.PART_LOCAL, local_order=2)
        S, D, _ = P.eval(np.array([0, 1, 2, 3 + node]))
        e = []
        for k, (t0, _) in enumerate(specs):
            s, d = _layer_brute(cv, (tx[k], ty[k]), t0, ds, alpha, dens)
            e.append((abs(S[k] - s), abs(D[k] - d)))
        # on-surface: D is the principal value (the average of the two sides)
        s, d = _layer_brute(cv, (bnd["x"][node], bnd["y"][node]), bnd["t"][node], ds, alpha, dens)
        e.append((abs(S[3] - s), abs(D[3] - d)))
        errs.append(e)
    errs = np.array(errs)                          # [ds][target][S, D]
    ratio = errs[0] / errs[1]
    assert np.all(ratio > 400), (errs, ratio)      # O(delta*^{5/2}): 1024; first order gives ~64
    assert errs[1, :, 0].max() < 5e-10 and errs[1, :, 1].max() < 2e-8, errs


_QC = dict(c0=1.0, cx=0.7, cy=-0.4, cxx=0.5, cxy=-0.3, cyy=0.8)


def _quad_f(x, y):
    c = _QC
    return c["c0"] + c["cx"] * x + c["cy"] * y + c["cxx"] * x * x + c["cxy"] * x * y + c["cyy"] * y * y


def _quad_jet(x, y):
    c = _QC
    return np.array([c["cx"] + 2 * c["cxx"] * x + c["cxy"] * y, c["cy"] + c["cxy"] * x + 2 * c["cyy"] * y,
                     np.full_like(x, 2 * c["cxx"]), np.full_like(x, c["cxy"]), np.full_like(x, 2 * c["cyy"])])


def _disk_local_volume(R, alpha, r0, th0, d):
    """int_0^d e^{-alpha^2 t} int_disk G_t(x - y) f(y) dy dt for the quadratic
    f of _QC at x = r0 (cos th0, sin th0): f in angular modes a_m(rho')
    e^{i m theta}, whose angular integrals against the heat kernel are
    modified Bessel functions I_m."""
    c = _QC

    def modes(rp):
        a1 = rp * (c["cx"] - 1j * c["cy"]) / 2
        a2 = rp * rp * (c["cxx"] - c["cyy"]) / 4 - 1j * rp * rp * c["cxy"] / 4
        return {0: c["c0"] + rp * rp * (c["cxx"] + c["cyy"]) / 2, 1: a1, -1: np.conj(a1), 2: a2, -2: np.conj(a2)}

    def inner(t):
        def g(rp):
            s = sum((a * np.exp(1j * m * th0)).real * sp.ive(abs(m), r0 * rp / (2 * t)) for m, a in modes(rp).items())
            return rp * s * math.exp(-(r0 - rp) ** 2 / (4 * t)) / (2 * t)
        lo, hi = max(0.0, r0 - 40 * math.sqrt(t)), min(R, r0 + 40 * math.sqrt(t))
        return integrate.quad(g, lo, hi, points=[r0] if lo < r0 < hi else None, epsabs=0, epsrel=1e-12,
                              limit=300)[0]
    return integrate.quad(lambda t: math.exp(-alpha ** 2 * t) * inner(t), 0, d, epsabs=0, epsrel=1e-11,
                          limit=300)[0]


def test_local_volume_order2_disk():
    """V_L with the second-order terms (Lemma 4.8, Corollary 4.10) for a
    quadratic f (its second-order Taylor expansion is exact) near the
    boundary of a disk and at a boundary node, against the local integral by
    Fourier-Bessel quadrature: error O(delta^{5/2})."""
    R, alpha = 0.5, 10.0
    bnd = synth.discretize([synth.Curve(r0=R)], 32)
    node = 5
    errs = []
    for d in (1e-3, 6.25e-5):
        sq = math.sqrt(d)
        tg = [(R - 1.2 * sq, 0.4), (R - 0.3 * sq, 1.9), (R - 3.0 * sq, 3.0)]
        tx = np.array([a * math.cos(b) for a, b in tg]); ty = np.array([a * math.sin(b) for a, b in tg])
        X = np.concatenate([tx, bnd["x"]]); Y = np.concatenate([ty, bnd["y"]])
        P = O.Problem(alpha, d, 0, bnd, targets=(tx, ty), inside=np.ones(3), on_surface=True, f_trg=_quad_f(X, Y),
                      f_jet=_quad_jet(X, Y), parts=O.PART_LOCAL, local_order=2)
        _, _, V = P.eval(np.array([0, 1, 2, 3 + node]))
        ref = [_disk_local_volume(R, alpha, a, b, d) for a, b in tg]
        ref.append(_disk_local_volume(R, alpha, R, math.atan2(bnd["y"][node], bnd["x"][node]), d))
        errs.append(np.abs(V - np.array(ref)))
    errs = np.array(errs)
    assert np.all(errs[0] / errs[1] > 400), errs   # O(delta^{5/2}): 1024
    assert errs[1].max() < 1e-10, errs
