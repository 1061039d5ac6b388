"""ctypes binding of libmhk.so (argument marshalling only).

Every step of the evaluation runs in the HIP library; this module only
converts numpy arrays and torch device tensors to the C ABI of
include/mhk.h.  Importing it without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmhk.so")

MHK_FP64, MHK_FP32 = 0, 1
PART_HISTORY, PART_LEVELS, PART_LOCAL, PART_ALL, PART_GEOMETRY = 1, 2, 4, 7, 8
NGL = 16


class Params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("tol", C.c_double), ("prec", C.c_int), ("J", C.c_int),
                ("delta", C.c_double), ("dx", C.c_double), ("batch", C.c_int),
                ("upsamp", C.c_double), ("wspread", C.c_int), ("local_order", C.c_int),
                ("lv_block", C.c_int), ("lv_bch", C.c_int), ("lv_persist", C.c_int), ("v_levels", C.c_int),
                ("in64", C.c_int)]


class Boundary(C.Structure):
    _fields_ = [("n_panels", C.c_int64), ("n_curves", C.c_int32), ("curve_panel_ofs", C.c_void_p),
                ("x", C.c_void_p), ("y", C.c_void_p), ("nx", C.c_void_p), ("ny", C.c_void_p),
                ("w", C.c_void_p), ("kappa", C.c_void_p)]


class Volume(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("w", C.c_void_p), ("group", C.c_int32),
                ("rule", C.c_void_p)]


class Targets(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("inside", C.c_void_p),
                ("on_surface", C.c_int)]


class Info(C.Structure):
    _fields_ = [("alpha", C.c_double), ("tol", C.c_double), ("delta", C.c_double), ("delta_star", C.c_double),
                ("J", C.c_int), ("prec", C.c_int), ("batch", C.c_int),
                ("kmax", C.c_double), ("period", C.c_double), ("n_fine", C.c_int64), ("wspread", C.c_int),
                ("band_layer", C.c_double), ("band_volume", C.c_double), ("level_radius", C.c_double * 8),
                ("n_boundary", C.c_int64), ("n_volume", C.c_int64), ("n_targets", C.c_int64),
                ("n_out", C.c_int64), ("device_bytes", C.c_int64),
                ("ms_spread", C.c_double), ("ms_fft", C.c_double), ("ms_multiply", C.c_double),
                ("ms_interp", C.c_double), ("ms_levels", C.c_double), ("ms_local", C.c_double),
                ("ms_total", C.c_double), ("history_truncated", C.c_int), ("n_noconv", C.c_int64),
                ("ms_geometry", C.c_double), ("ms_plan", C.c_double * 6)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name in ("level_radius", "ms_plan") else v
        return d


class NysInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("alpha", C.c_double), ("device_bytes", C.c_int64), ("ms_assemble", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("resid", C.c_double), ("ms_eval", C.c_double),
                ("ms_gmres", C.c_double), ("ms_total", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


EXPORTS = ["mhk_resolve_params", "mhk_plan_create", "mhk_plan_footprint", "mhk_eval", "mhk_eval_S",
           "mhk_eval_D", "mhk_eval_V", "mhk_eval_parts", "mhk_eval_batch", "mhk_plan_f_targets", "mhk_plan_capture", "mhk_plan_launch_graph",
           "mhk_plan_set_timing", "mhk_plan_info", "mhk_plan_destroy", "mhk_last_error",
           "mhk_nystrom_create", "mhk_nystrom_apply", "mhk_nystrom_solve", "mhk_nystrom_solve_noalloc",
           "mhk_solve_dirichlet",
           "mhk_solve_neumann", "mhk_heat_step", "mhk_nystrom_info", "mhk_nystrom_destroy"]
_VOID = ("mhk_plan_destroy", "mhk_last_error", "mhk_nystrom_destroy")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libmhk.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.mhk_resolve_params.argtypes = [P(Params), P(Info)]
        L.mhk_plan_create.argtypes = [P(Params), P(Boundary), P(Volume), P(Targets), C.c_void_p, P(C.c_void_p)]
        L.mhk_plan_footprint.argtypes = [P(Params), P(Boundary), P(Volume), P(Targets), P(C.c_int64)]
        L.mhk_eval.argtypes = [C.c_void_p] + [C.c_void_p] * 7
        L.mhk_eval_S.argtypes = [C.c_void_p] * 3
        L.mhk_eval_D.argtypes = [C.c_void_p] * 3
        L.mhk_eval_V.argtypes = [C.c_void_p] * 4
        L.mhk_eval_parts.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 7
        L.mhk_eval_batch.argtypes = [C.c_void_p, C.c_int, C.c_int] + [C.c_void_p] * 7
        L.mhk_plan_f_targets.argtypes = [C.c_void_p] * 3
        L.mhk_plan_capture.argtypes = [C.c_void_p, C.c_int] + [C.c_void_p] * 7
        L.mhk_plan_launch_graph.argtypes = [C.c_void_p]
        L.mhk_plan_set_timing.argtypes = [C.c_void_p, C.c_int]
        L.mhk_plan_info.argtypes = [C.c_void_p, P(Info)]
        L.mhk_plan_destroy.argtypes = [C.c_void_p]
        L.mhk_plan_destroy.restype = None
        L.mhk_last_error.restype = C.c_char_p
        d, vp, i = C.c_double, C.c_void_p, C.c_int
        L.mhk_nystrom_create.argtypes = [d, P(Boundary), vp, P(vp)]
        L.mhk_nystrom_apply.argtypes = [vp, d, vp, vp]
        L.mhk_nystrom_solve.argtypes = [vp, d, vp, vp, d, i, i, P(SolveInfo)]
        L.mhk_nystrom_solve_noalloc.argtypes = [vp, d, vp, vp, d, i, i, P(SolveInfo)]
        L.mhk_solve_dirichlet.argtypes = [vp, vp, vp, vp, vp, d, i, i, vp, vp, P(SolveInfo)]
        L.mhk_solve_neumann.argtypes = [vp, vp, vp, vp, vp, d, i, i, vp, vp, P(SolveInfo)]
        L.mhk_heat_step.argtypes = [vp, vp, vp, vp, vp, d, i, i, vp, vp, P(SolveInfo)]
        L.mhk_nystrom_info.argtypes = [vp, P(NysInfo)]
        L.mhk_nystrom_destroy.argtypes = [vp]
        L.mhk_nystrom_destroy.restype = None
        for name in EXPORTS:
            if name not in _VOID:
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class MhkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mhk error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise MhkError(rc, lib().mhk_last_error().decode())


def make_params(alpha, tol, prec=MHK_FP64, J=3, delta=0.0, dx=0.0, batch=1, upsamp=0.0, wspread=0, local_order=1,
                lv_block=0, lv_bch=0, in64=0, v_levels=0, lv_persist=0):
    return Params(float(alpha), float(tol), int(prec), int(J), float(delta), float(dx), int(batch),
                  float(upsamp), int(wspread), int(local_order), int(lv_block), int(lv_bch), int(lv_persist),
                  int(v_levels), int(in64))


def resolve_params(**kw):
    info = Info()
    _check(lib().mhk_resolve_params(C.byref(make_params(**kw)), C.byref(info)))
    return info.as_dict()


class _Keep:
    def __init__(self):
        self.arrays = []

    def f64(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self.arrays.append(a)
        return a.ctypes.data

    def typed(self, a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        self.arrays.append(a)
        return a.ctypes.data


def _structs(boundary, volume, targets, on_surface, keep):
    b = boundary
    nb = len(b["x"])
    if nb % NGL:
        raise ValueError("boundary size must be a multiple of 16")
    ofs = np.asarray(b.get("curve_panel_ofs", [0, nb // NGL]), dtype=np.int64)
    B = Boundary(nb // NGL, len(ofs) - 1, keep.typed(ofs, np.int64), keep.f64(b["x"]), keep.f64(b["y"]),
                 keep.f64(b["nx"]), keep.f64(b["ny"]), keep.f64(b["w"]), keep.f64(b["kappa"]))
    if volume is not None and len(volume["x"]) > 0:
        rule = volume.get("rule")
        V = Volume(len(volume["x"]), keep.f64(volume["x"]), keep.f64(volume["y"]), keep.f64(volume["w"]),
                   int(volume.get("group", 0)), None if rule is None else keep.f64(np.asarray(rule).ravel()))
    else:
        V = Volume(0, None, None, None, 0, None)
    if targets is not None:
        tx, ty, ins = targets
        T = Targets(len(tx), keep.f64(tx), keep.f64(ty),
                    None if ins is None else keep.typed(np.asarray(ins).astype(np.int8), np.int8),
                    int(bool(on_surface)))
    else:
        T = Targets(0, None, None, None, int(bool(on_surface)))
    return B, V, T


def footprint(params, boundary, volume=None, targets=None, on_surface=False):
    keep = _Keep()
    B, V, T = _structs(boundary, volume, targets, on_surface, keep)
    out = C.c_int64(0)
    _check(lib().mhk_plan_footprint(C.byref(params), C.byref(B), C.byref(V), C.byref(T), C.byref(out)))
    return int(out.value)


class Plan:
    """A resident evaluation plan on the current torch HIP stream.

    boundary: dict of host arrays x, y, nx, ny, w, kappa (16 Gauss-Legendre
    nodes per panel, panel contiguous) and curve_panel_ofs; volume: dict x, y,
    w or None; targets: (x, y, inside) host arrays, inside None to have the
    plan compute it.
    """

    def __init__(self, params: Params, boundary, volume=None, targets=None, on_surface=False, stream=None):
        import torch
        self.params = params
        keep = _Keep()
        B, V, T = _structs(boundary, volume, targets, on_surface, keep)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        _check(lib().mhk_plan_create(C.byref(params), C.byref(B), C.byref(V), C.byref(T),
                                     C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h
        self.nb = int(B.n_panels) * NGL
        self.nv = int(V.n)
        self.nt = int(T.n)
        self.n_out = self.nt + (self.nb if on_surface else 0)
        self.batch = int(params.batch)
        self.dtype = torch.float64 if params.prec == MHK_FP64 else torch.float32
        # densities and f as given by the caller (double for FP32 plans with in64)
        self.in_dtype = torch.float64 if (params.prec == MHK_FP64 or params.in64) else torch.float32
        # f at the targets: the value, or (local_order 2) the value, gradient and Hessian
        self.f_rows = 6 if int(params.local_order) == 2 else 1

    def close(self):
        if getattr(self, "_h", None):
            lib().mhk_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = Info()
        _check(lib().mhk_plan_info(self._h, C.byref(i)))
        return i.as_dict()

    def set_timing(self, on=True):
        _check(lib().mhk_plan_set_timing(self._h, int(bool(on))))

    def _dev(self, t, n, nb=None, dtype=None):
        import torch
        if t is None:
            return None
        nb = self.batch if nb is None else nb
        dtype = self.in_dtype if dtype is None else dtype
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
            raise TypeError(f"expected a contiguous {dtype} device tensor")
        if t.numel() != nb * n:
            raise ValueError(f"expected {nb} x {n} values, got {t.numel()}")
        return t

    def _outs(self, out, ins, nb=None):
        """Output tensors: allocated when out is None, else checked like the
        inputs (a short or mistyped output would be written past its end)."""
        import torch
        nb = self.batch if nb is None else nb
        shape = (nb, self.n_out)
        if out is None:
            return tuple(torch.empty(shape, dtype=self.dtype, device="cuda") if x is not None else None
                         for x in ins)
        if len(out) != 3:
            raise ValueError("out must be a (S, D, V) tuple")
        for x, o, name in zip(ins, out, ("S", "D", "V")):
            if x is None:
                continue
            if o is None:
                raise ValueError(f"out[{name}] is missing for a given input")
            self._dev(o, self.n_out, nb, self.dtype)
        return tuple(out)

    def _streams(self):
        """(caller's current stream, whether it differs from the plan's)."""
        import torch
        cur = torch.cuda.current_stream()
        return cur, cur.cuda_stream != self.stream.cuda_stream

    def capture(self, sigma=None, mu=None, f_vol=None, f_trg=None, parts=PART_ALL, out=None):
        """Record one evaluation bound to these tensors into a HIP graph;
        returns the output tensors the graph writes.  replay() runs it on the
        plan's stream; the caller keeps the bound tensors alive."""
        sigma = self._dev(sigma, self.nb)
        mu = self._dev(mu, self.nb)
        f_vol = self._dev(f_vol, self.nv)
        f_trg = self._dev(f_trg, self.f_rows * self.n_out)
        out = self._outs(out, (sigma, mu, f_vol))
        cur, other = self._streams()
        if other:
            # the capture synchronises the plan's stream; the inputs may still
            # be written on the caller's stream
            cur.synchronize()
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        _check(lib().mhk_plan_capture(self._h, int(parts), ptr(sigma), ptr(mu), ptr(f_vol), ptr(f_trg),
                                      ptr(out[0]), ptr(out[1]), ptr(out[2])))
        self._bound = (sigma, mu, f_vol, f_trg, out)
        return out

    def f_targets(self, f_vol, out=None):
        """f at the targets as reconstructed from the volume triangles (the
        f_trg an eval uses when given none): [batch, rows, n_out]."""
        import torch
        f_vol = self._dev(f_vol, self.nv)
        if out is None:
            out = torch.empty((self.batch, self.f_rows, self.n_out), dtype=self.in_dtype, device="cuda")
        self._dev(out, self.f_rows * self.n_out, None, self.in_dtype)
        cur, other = self._streams()
        if other:
            self.stream.wait_stream(cur)
        _check(lib().mhk_plan_f_targets(self._h, C.c_void_p(f_vol.data_ptr()), C.c_void_p(out.data_ptr())))
        if other:
            cur.wait_stream(self.stream)
        return out

    def replay(self):
        _check(lib().mhk_plan_launch_graph(self._h))

    def eval(self, sigma=None, mu=None, f_vol=None, f_trg=None, parts=PART_ALL, out=None, join=True, nbatch=None):
        """Returns (S, D, V) device tensors [batch, n_out] (None where not requested).
        nbatch (1..batch): evaluate only that many densities (inputs and
        outputs [nbatch, ...]; mhk_eval_batch).

        The work runs on the plan's stream.  When the caller's current stream
        is another one, the plan's stream first waits for it (the inputs may
        still be written there), the tensors are marked as used on the plan's
        stream, and with join=True the caller's stream then waits for the
        evaluation, so that the outputs can be used on it directly; join=False
        leaves that wait to the caller (several plans overlapping)."""
        nb = self.batch if nbatch is None else int(nbatch)
        if not 1 <= nb <= self.batch:
            raise ValueError(f"nbatch must be in [1, {self.batch}]")
        sigma = self._dev(sigma, self.nb, nb)
        mu = self._dev(mu, self.nb, nb)
        f_vol = self._dev(f_vol, self.nv, nb)
        f_trg = self._dev(f_trg, self.f_rows * self.n_out, nb)
        out = self._outs(out, (sigma, mu, f_vol), nb)
        cur, other = self._streams()
        if other:
            self.stream.wait_stream(cur)
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        if nb == self.batch:
            _check(lib().mhk_eval_parts(self._h, int(parts), ptr(sigma), ptr(mu), ptr(f_vol), ptr(f_trg),
                                        ptr(out[0]), ptr(out[1]), ptr(out[2])))
        else:
            _check(lib().mhk_eval_batch(self._h, nb, int(parts), ptr(sigma), ptr(mu), ptr(f_vol), ptr(f_trg),
                                        ptr(out[0]), ptr(out[1]), ptr(out[2])))
        if other:
            for t in (sigma, mu, f_vol, f_trg) + tuple(out):
                if t is not None:
                    t.record_stream(self.stream)
            if join:
                cur.wait_stream(self.stream)
        return out


def _f64_dev(t, n, what):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{what} must be a contiguous float64 device tensor")
    if t.numel() != n:
        raise ValueError(f"{what}: expected {n} values, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Nystrom:
    """The dense Nystrom matrix K of the double-layer operator on the boundary
    nodes, resident on the device, with its product and GMRES solve."""

    def __init__(self, alpha, boundary, stream=None):
        import torch
        keep = _Keep()
        B, _, _ = _structs(boundary, None, None, False, keep)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.alpha = float(alpha)
        self.n = int(B.n_panels) * NGL
        h = C.c_void_p()
        _check(lib().mhk_nystrom_create(self.alpha, C.byref(B), C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().mhk_nystrom_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = NysInfo()
        _check(lib().mhk_nystrom_info(self._h, C.byref(i)))
        return {name: getattr(i, name) for name, _ in i._fields_}

    def apply(self, x, shift=0.0, out=None):
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(lib().mhk_nystrom_apply(self._h, float(shift), _f64_dev(x, self.n, "x"), _f64_dev(out, self.n, "y")))
        return out

    def solve(self, rhs, shift, tol=1e-12, restart=60, maxit=500, out=None, noalloc=False):
        """GMRES solve of (shift I + K) x = rhs.  noalloc=True calls
        mhk_nystrom_solve_noalloc (workspace from the library's fixed scratch
        array; out must then be given, and restart <= 64)."""
        import torch
        if out is None:
            if noalloc:
                raise ValueError("noalloc=True needs the output vector")
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        info = SolveInfo()
        fn = lib().mhk_nystrom_solve_noalloc if noalloc else lib().mhk_nystrom_solve
        _check(fn(self._h, float(shift), _f64_dev(rhs, self.n, "rhs"), _f64_dev(out, self.n, "x"), float(tol),
                  int(restart), int(maxit), C.byref(info)))
        return out, info.as_dict()


def _solve(kind, plan, nys, g, f_vol, f_trg, tol, restart, maxit):
    import torch
    dens = torch.empty(plan.nb, dtype=torch.float64, device="cuda")
    u = torch.empty(plan.n_out, dtype=torch.float64, device="cuda")
    fv = None if f_vol is None else _f64_dev(f_vol, plan.nv, "f_vol")
    ft = None if f_trg is None else _f64_dev(f_trg, plan.n_out, "f_trg")
    info = SolveInfo()
    fn = lib().mhk_solve_dirichlet if kind == "dirichlet" else lib().mhk_solve_neumann
    _check(fn(plan._h, nys._h, _f64_dev(g, plan.nb, "g"), fv, ft, float(tol), int(restart), int(maxit),
              C.c_void_p(dens.data_ptr()), C.c_void_p(u.data_ptr()), C.byref(info)))
    return dens, u, info.as_dict()


def solve_dirichlet(plan, nys, g, f_vol=None, f_trg=None, tol=1e-12, restart=60, maxit=500):
    """Returns (mu, u, info): layer density and u at every output of the plan."""
    return _solve("dirichlet", plan, nys, g, f_vol, f_trg, tol, restart, maxit)


def solve_neumann(plan, nys, g, f_vol=None, f_trg=None, tol=1e-12, restart=60, maxit=500):
    """Returns (u_b, u, info): boundary values and u at every output of the plan."""
    return _solve("neumann", plan, nys, g, f_vol, f_trg, tol, restart, maxit)


def heat_step(plan, nys, u_n, g_next, F=None, tol=1e-12, restart=60, maxit=500, out=None):
    """One implicit-Euler step of the heat equation with time step
    1/alpha^2 (the plan's targets are its volume nodes).  u_n, F: [n_out]
    over the volume nodes then the boundary nodes; g_next: [N_B].  Returns
    (u_next, mu, info)."""
    import torch
    u = torch.empty(plan.n_out, dtype=torch.float64, device="cuda") if out is None else out
    mu = torch.empty(plan.nb, dtype=torch.float64, device="cuda")
    info = SolveInfo()
    _check(lib().mhk_heat_step(plan._h, nys._h, _f64_dev(u_n, plan.n_out, "u_n"),
                               None if F is None else _f64_dev(F, plan.n_out, "F"),
                               _f64_dev(g_next, plan.nb, "g_next"), float(tol), int(restart), int(maxit),
                               _f64_dev(u, plan.n_out, "u_next"), C.c_void_p(mu.data_ptr()), C.byref(info)))
    return u, mu, info.as_dict()
