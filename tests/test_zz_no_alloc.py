"""mhk_nystrom_solve_noalloc, the GMRES solve whose workspace is the
library's fixed device scratch array, against mhk_nystrom_solve on the same
Nystrom matrices, through the C ABI: two calls in a row, the second on a
smaller boundary (the scratch then holds the first call's larger contents),
at the bar of the solves (the same kernels in the same order: agreement to
rounding, 1e-14 of max |x|, and the same iteration count)."""
import ctypes as C

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(w, alpha, seed):
    import paper_2606_28865_amd as M
    nys = M.Nystrom(alpha, w.boundary)
    g = np.random.default_rng(seed)
    rhs = torch.as_tensor(g.standard_normal(nys.n), dtype=torch.float64, device="cuda")
    return nys, rhs


def _solve_raw(nys, rhs, x, restart, noalloc):
    from paper_2606_28865_amd import _lib as L
    info = L.SolveInfo()
    fn = L.lib().mhk_nystrom_solve_noalloc if noalloc else L.lib().mhk_nystrom_solve
    rc = fn(nys._h, -0.5, C.c_void_p(rhs.data_ptr()), C.c_void_p(x.data_ptr()), 1e-12, restart, 400,
            C.byref(info))
    return rc, info


def test_noalloc_solve_matches_allocating_solve():
    from paper_2606_28865_amd import _lib as L
    big = synth.multibody(cfg=21, n_bodies=3, n_boundary=4096, n_volume=20000, n_targets=10, box=0.6)
    small = synth.config0()
    for name, w, alpha, restart in (("4096 nodes", big, 10.0, 40), ("512 nodes", small, 3.0, 20)):
        print(f"case noalloc GMRES {name} alpha={alpha} restart={restart}", flush=True)
        nys, rhs = _case(w, alpha, seed=len(name))
        x_ref = torch.empty_like(rhs)
        x_na = torch.full_like(rhs, float("nan"))
        rc, info_ref = _solve_raw(nys, rhs, x_ref, restart, noalloc=False)
        assert rc == 0, L.lib().mhk_last_error()
        rc, info_na = _solve_raw(nys, rhs, x_na, restart, noalloc=True)
        assert rc == 0, L.lib().mhk_last_error()
        torch.cuda.synchronize()
        assert info_na.converged == 1 and info_ref.converged == 1
        assert info_na.iters == info_ref.iters
        err = float((x_na - x_ref).abs().max() / x_ref.abs().max())
        print(f"{name}: {info_na.iters} iterations, residual {info_na.resid:.2e}, max diff {err:.2e}", flush=True)
        assert err <= 1e-14
        # restart beyond the fixed scratch's limit: rejected before any work
        rc, _ = _solve_raw(nys, rhs, x_na, 65, noalloc=True)
        assert rc == -1          # MHK_EINVAL
        nys.close()
