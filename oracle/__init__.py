"""CPU FP64 oracle for the kernel-split modified-Helmholtz potentials.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product package.  All arithmetic
lives in mhk_oracle.c; this module only marshals numpy arrays through ctypes.

The oracle evaluates the same split sums as the fast method (Section 2.1:
history part for t > delta, J dyadic difference-kernel levels, local
asymptotic part) with the history and level parts summed directly in real
space over every source.  See mhk_oracle.c for the readings of the paper it
follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_mhk.so")
_lib = None

NGL = 16
PART_HISTORY, PART_LEVELS, PART_LOCAL = 1, 2, 4
PART_ALL = 7


class _Problem(C.Structure):
    _fields_ = [
        ("alpha", C.c_double), ("delta", C.c_double), ("J", C.c_int), ("parts", C.c_int),
        ("n_panels", C.c_int64),
        ("bx", C.c_void_p), ("by", C.c_void_p), ("bnx", C.c_void_p), ("bny", C.c_void_p),
        ("bw", C.c_void_p), ("bkappa", C.c_void_p),
        ("panel_prev", C.c_void_p), ("panel_next", C.c_void_p),
        ("n_vol", C.c_int64), ("vx", C.c_void_p), ("vy", C.c_void_p), ("vw", C.c_void_p),
        ("n_trg", C.c_int64), ("tx", C.c_void_p), ("ty", C.c_void_p), ("inside", C.c_void_p),
        ("on_surface", C.c_int),
        ("sigma", C.c_void_p), ("mu", C.c_void_p), ("f_vol", C.c_void_p), ("f_trg", C.c_void_p),
        ("local_order", C.c_int), ("f_jet", C.c_void_p),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "mhk_oracle.c"))):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        d, i = C.c_double, C.c_int
        for name in ("or_GH", "or_GHD", "or_GR"):
            f = getattr(L, name); f.restype = d; f.argtypes = [d, d, d]
        for name in ("or_KS", "or_KD"):
            f = getattr(L, name); f.restype = d; f.argtypes = [d, d, d, i]
        L.or_local_coeffs.restype = None
        L.or_local_coeffs.argtypes = [d, d, C.c_void_p]
        L.or_gl_rule.restype = None
        L.or_gl_rule.argtypes = [i, C.c_void_p, C.c_void_p]
        L.or_refine_level.restype = i
        L.or_refine_level.argtypes = [C.POINTER(_Problem), i] + [C.c_void_p] * 7
        L.or_closest_point.restype = i
        L.or_closest_point.argtypes = [C.POINTER(_Problem), d, d, C.c_void_p]
        L.or_level_sum_S.restype = None
        L.or_level_sum_S.argtypes = [d, d, i, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_eval.restype = i
        L.or_eval.argtypes = [C.POINTER(_Problem), C.c_void_p, C.c_int64,
                              C.c_void_p, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _vec(f):
    return np.vectorize(f, otypes=[float])


def GH(r, alpha, delta):
    """History kernel int_delta^inf H dt at distance r."""
    return _vec(lambda x: lib().or_GH(float(x), alpha, delta))(r)


def GHD(r, alpha, delta):
    """Double-layer history factor int_delta^inf H/(2t) dt."""
    return _vec(lambda x: lib().or_GHD(float(x), alpha, delta))(r)


def GR(r, alpha, d):
    """Real-space part int_0^d H dt."""
    return _vec(lambda x: lib().or_GR(float(x), alpha, d))(r)


def KS(r, alpha, delta, j):
    return _vec(lambda x: lib().or_KS(float(x), alpha, delta, int(j)))(r)


def KD(r, alpha, delta, j):
    return _vec(lambda x: lib().or_KD(float(x), alpha, delta, int(j)))(r)


LOCAL_NAMES = ["Phim", "Phip", "Z", "P0", "P1", "P2", "P3", "Q0", "Q1",
               "U0", "U1", "U2", "U3", "U4", "lam", "W0", "W1"]


def level_sum_S(alpha, delta, j, sx, sy, q, tx, ty):
    """sum_s q_s K_j^S(|x_t - y_s|) at every target, direct."""
    sx, sy, q, tx, ty = (np.ascontiguousarray(a, dtype=np.float64) for a in (sx, sy, q, tx, ty))
    out = np.zeros(len(tx))
    lib().or_level_sum_S(float(alpha), float(delta), int(j), len(sx), sx.ctypes.data, sy.ctypes.data,
                         q.ctypes.data, len(tx), tx.ctypes.data, ty.ctypes.data, out.ctypes.data)
    return out


def local_coeffs(c1, c2):
    """Coefficients of Lemmas 4.1/4.5/4.8 as a dict (evaluated in __float128)."""
    out = np.zeros(len(LOCAL_NAMES))
    lib().or_local_coeffs(float(c1), float(c2), out.ctypes.data)
    return dict(zip(LOCAL_NAMES, out))


def gl_rule(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().or_gl_rule(n, x.ctypes.data, w.ctypes.data)
    return x, w


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Problem:
    """Holds numpy arrays alive and exposes the C problem struct.

    boundary: dict with x, y, nx, ny, w, kappa (panel-contiguous, 16 nodes per
    panel, counter-clockwise, outward normal) and panel_prev/panel_next.
    """

    def __init__(self, alpha, delta, J, boundary, volume=None, targets=None,
                 inside=None, on_surface=False, sigma=None, mu=None, f_vol=None,
                 f_trg=None, parts=PART_ALL, local_order=1, f_jet=None):
        """local_order 1 keeps the local expansions to first order (Section
        4.1); 2 adds their printed second-order terms, with f_jet the
        gradient and Hessian of f at the targets, [5][n_out] = f_x, f_y,
        f_xx, f_xy, f_yy (needed for V)."""
        self._keep = []
        p = _Problem()
        p.alpha, p.delta, p.J, p.parts = float(alpha), float(delta), int(J), int(parts)
        b = boundary
        nb = len(b["x"])
        assert nb % NGL == 0
        p.n_panels = nb // NGL
        for key, field in (("x", "bx"), ("y", "by"), ("nx", "bnx"), ("ny", "bny"),
                           ("w", "bw"), ("kappa", "bkappa")):
            setattr(p, field, self._ptr(_f64(b[key])))
        p.panel_prev = self._ptr(np.ascontiguousarray(b["panel_prev"], dtype=np.int64))
        p.panel_next = self._ptr(np.ascontiguousarray(b["panel_next"], dtype=np.int64))
        if volume is not None:
            p.n_vol = len(volume["x"])
            p.vx, p.vy, p.vw = (self._ptr(_f64(volume[k])) for k in ("x", "y", "w"))
        if targets is not None:
            tx, ty = targets
            p.n_trg = len(tx)
            p.tx, p.ty = self._ptr(_f64(tx)), self._ptr(_f64(ty))
            if inside is not None:
                p.inside = self._ptr(np.ascontiguousarray(inside, dtype=np.int8))
        p.on_surface = int(bool(on_surface))
        p.sigma = self._ptr(_f64(sigma)); p.mu = self._ptr(_f64(mu))
        p.f_vol = self._ptr(_f64(f_vol)); p.f_trg = self._ptr(_f64(f_trg))
        p.local_order = int(local_order)
        if f_jet is not None:
            f_jet = np.ascontiguousarray(f_jet, dtype=np.float64)
            assert f_jet.shape == (5, int(p.n_trg) + (nb if on_surface else 0)), f_jet.shape
        p.f_jet = self._ptr(f_jet)
        self.c = p
        self.n_b = nb
        self.n_out = int(p.n_trg) + (nb if on_surface else 0)

    def _ptr(self, a):
        if a is None:
            return None
        self._keep.append(a)
        return a.ctypes.data

    def eval(self, subset=None):
        """Returns (S, D, V) for all targets, or for target indices `subset`."""
        if subset is not None:
            sub = np.ascontiguousarray(subset, dtype=np.int64)
            n = len(sub); sp = sub.ctypes.data
        else:
            n = self.n_out; sp = None
        S, D, V = np.zeros(n), np.zeros(n), np.zeros(n)
        rc = lib().or_eval(C.byref(self.c), sp, n, S.ctypes.data, D.ctypes.data, V.ctypes.data)
        assert rc == 0
        return S, D, V

    def refine(self, j):
        n = self.n_b * (1 << j)
        arrs = [np.zeros(n) for _ in range(7)]
        lib().or_refine_level(C.byref(self.c), j, *[a.ctypes.data for a in arrs])
        return dict(zip(["x", "y", "nx", "ny", "w", "sigma", "mu"], arrs))

    def closest(self, px, py):
        out = np.zeros(5)
        lib().or_closest_point(C.byref(self.c), float(px), float(py), out.ctypes.data)
        return {"panel": int(out[0]), "t": out[1], "x0": out[2], "y0": out[3], "r": out[4]}
