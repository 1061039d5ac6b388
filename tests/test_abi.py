"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/mhk.h, applies the parameter rule of
Section 6.4 and rejects invalid arguments; without the library the
binding raises."""
import math
import os
import re

import numpy as np
import pytest

import paper_2606_28865_amd as M
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mhk.h")).read()
    return sorted(set(re.findall(r"\b(mhk_[a-z_A-Z]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = M.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


def _golden():
    vals = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "hilbert_chain.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split("=")
            vals[k.strip()] = float(v)
    return vals


def test_parameter_rule_hilbert_chain():
    """Section 6.4: dx ~ 2.5e-3, k_max = 0.9 pi/dx ~ 1141, delta ~ 1.06e-5,
    delta* ~ 1.66e-7 with J = 3 and eps = 1e-6, alpha = 10."""
    g = _golden()
    dx = 0.9 * math.pi / g["kmax"]
    assert dx == pytest.approx(g["dx"], rel=0.02)
    info = M.resolve_params(alpha=g["alpha"], tol=g["eps"], dx=dx, J=int(g["J"]))
    assert info["delta"] == pytest.approx(g["delta"], rel=5e-3)
    assert info["delta_star"] == pytest.approx(g["delta_star"], rel=5e-3)
    # the history cut-off uses the stricter double-layer rule (eq. (kmax_dlp))
    k, d, a, eps = info["kmax"], info["delta"], g["alpha"], g["eps"]
    assert k * math.exp(-d * (a * a + k * k)) == pytest.approx(eps, rel=1e-8)


def test_bands_and_levels():
    info = M.resolve_params(alpha=10.0, tol=1e-10, delta=1e-3, J=3)
    ds = 1e-3 / 64
    assert info["band_layer"] == pytest.approx(math.sqrt(ds) * (12 + 2 * 10 * math.sqrt(ds)), rel=1e-14)
    assert info["band_volume"] == pytest.approx(math.sqrt(1e-3) * (12 + 20 * math.sqrt(1e-3)), rel=1e-14)
    r = info["level_radius"]
    assert r[0] / r[1] == pytest.approx(2.0) and r[1] / r[2] == pytest.approx(2.0)
    # the history vanishes when delta alpha^2 >= ln(1/eps) (Section 5.2)
    assert M.resolve_params(alpha=300.0, tol=1e-6, delta=1e-3)["kmax"] == 0.0


def test_history_rule_shared_by_precisions():
    """The history cut-off and window width follow the requested tolerance
    at both precisions, so FP32 and FP64 plans of one problem share them."""
    for alpha, tol in ((30.0, 1e-6), (3.0, 1e-6), (10.0, 1e-7)):
        a = M.resolve_params(alpha=alpha, tol=tol, prec=M.MHK_FP64, delta=1e-4)
        b = M.resolve_params(alpha=alpha, tol=tol, prec=M.MHK_FP32, delta=1e-4)
        assert a["kmax"] == b["kmax"] and a["wspread"] == b["wspread"]
    # a tighter tolerance widens the window
    w6 = M.resolve_params(alpha=10.0, tol=1e-6, prec=M.MHK_FP32, delta=1e-4)["wspread"]
    w10 = M.resolve_params(alpha=10.0, tol=1e-10, prec=M.MHK_FP64, delta=1e-4)["wspread"]
    assert w10 > w6


@pytest.mark.parametrize("kw", [dict(alpha=-1.0, tol=1e-6, delta=1e-3), dict(alpha=1.0, tol=1e-1, delta=1e-3),
                                dict(alpha=1.0, tol=1e-6), dict(alpha=1.0, tol=1e-6, delta=1e-3, J=9),
                                dict(alpha=1.0, tol=1e-6, delta=1e-3, batch=0),
                                dict(alpha=1.0, tol=1e-6, delta=1e-3, prec=3),
                                dict(alpha=1.0, tol=1e-6, delta=1e-3, wspread=2),
                                dict(alpha=float("nan"), tol=1e-6, delta=1e-3),
                                dict(alpha=10.0, tol=1e-10, prec=1, delta=1e-3)])
def test_invalid_params_rejected(kw):
    with pytest.raises(M.MhkError) as e:
        M.resolve_params(**kw)
    assert e.value.code == -1


def test_footprint_and_input_validation():
    w = synth.config0()
    prm = M.make_params(alpha=10.0, tol=1e-10, dx=w.dx)
    nbytes = M.footprint(prm, w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True)
    assert nbytes > 0
    b2 = dict(w.boundary)
    b2["x"] = w.boundary["x"].copy()
    b2["x"][3] = np.nan
    with pytest.raises(M.MhkError):
        M.footprint(prm, b2, w.volume, (w.tx, w.ty, w.inside), on_surface=True)
    with pytest.raises(M.MhkError):
        M.footprint(prm, w.boundary, w.volume, None, on_surface=False)
    b3 = dict(w.boundary)
    b3["curve_panel_ofs"] = np.array([0, 5])
    with pytest.raises(M.MhkError):
        M.footprint(prm, b3, w.volume, (w.tx, w.ty, w.inside), on_surface=True)


def test_nystrom_argument_validation():
    """Argument checks of the boundary-integral entry points happen on the host
    before any device call."""
    import ctypes as C
    from paper_2606_28865_amd import _lib
    w = synth.config0()
    keep = _lib._Keep()
    B, _, _ = _lib._structs(w.boundary, None, None, False, keep)
    L = M.lib()
    h = C.c_void_p()
    for alpha in (0.0, -1.0, float("nan")):
        assert L.mhk_nystrom_create(alpha, C.byref(B), None, C.byref(h)) == -1
        assert not h.value
    assert L.mhk_nystrom_create(10.0, None, None, C.byref(h)) == -1
    assert L.mhk_nystrom_create(10.0, C.byref(B), None, None) == -1
    info = _lib.SolveInfo()
    assert L.mhk_nystrom_solve(None, 0.5, None, None, 1e-10, 30, 100, C.byref(info)) == -1
    assert L.mhk_nystrom_apply(None, 0.5, None, None) == -1
    assert L.mhk_solve_dirichlet(None, None, None, None, None, 1e-10, 30, 100, None, None, C.byref(info)) == -1
    assert L.mhk_solve_neumann(None, None, None, None, None, 1e-10, 30, 100, None, None, C.byref(info)) == -1
    L.mhk_nystrom_destroy(None)


def test_missing_library_fails_loudly():
    """Without the built library the binding raises on first use: there is
    no other path to the results."""
    import subprocess
    import sys
    code = ("import paper_2606_28865_amd._lib as L\n"
            "L.LIB_PATH = '/nonexistent/libmhk.so'\n"
            "try:\n"
            "    L.resolve_params(alpha=10.0, tol=1e-6, delta=1e-3)\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    raise SystemExit('no error')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "not built" in r.stdout
