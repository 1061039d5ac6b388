"""f at the targets from the volume quadrature (volume nodes in groups of
six per triangle): the plan's reconstruction against the oracle's
(oracle/fjets.py), and the potentials with f_trg omitted against the
oracle fed the oracle's reconstruction, FP64 at 1e-10, first and second
order (f's gradient and Hessian from the same quadratics)."""
import numpy as np
import pytest

import oracle as O
import synth
from helpers import rel_err, small_multibody, stratified_subset
from oracle import fjets

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _plan(w, alpha, **kw):
    import paper_2606_28865_amd as M
    return M.Plan(M.make_params(alpha=alpha, tol=kw.pop("tol", TOL), dx=w.dx, **kw), w.boundary, w.volume,
                  (w.tx, w.ty, w.inside), on_surface=True)


def _oracle(w, alpha, delta, ftrg, order=1, subset=None):
    P = O.Problem(alpha, delta, 3, w.boundary, volume=w.volume, targets=(w.tx, w.ty), inside=w.inside,
                  on_surface=True, sigma=w.sigma, mu=w.mu, f_vol=w.f_vol, f_trg=ftrg[0],
                  f_jet=ftrg[1:] if order == 2 else None, local_order=order)
    return P.eval(subset)


@pytest.mark.parametrize("order", [1, 2])
def test_reconstruction_matches_oracle(order):
    w = synth.config0()
    assert w.volume["group"] == 6
    print(f"case f at targets config0 order {order}", flush=True)
    plan = _plan(w, 10.0, local_order=order)
    got = plan.f_targets(_dev(w.f_vol)).cpu().numpy()[0]
    ref = fjets.f_at_targets(w.volume, w.f_vol, w.tx, w.ty, w.inside, w.boundary, rows=6 if order == 2 else 1)
    for r in range(got.shape[0]):
        e = np.abs(got[r] - ref[r]).max() / np.abs(ref[r]).max()
        print(f"row {r}: {e:.2e}", flush=True)
        assert e < 1e-10, (r, e)
    # the analytic source: the reconstruction is accurate to O(h^3)
    f_exact = w.f_trg
    need = np.concatenate([w.inside.astype(bool), np.ones(w.n_b, bool)])
    assert np.abs(got[0][need] - f_exact[need]).max() < 1e-3 * np.abs(f_exact).max()


@pytest.mark.parametrize("alpha", [10.0, 3.0])
def test_eval_without_f_trg_config0(alpha):
    w = synth.config0()
    print(f"case eval without f_trg config0 alpha={alpha}", flush=True)
    plan = _plan(w, alpha)
    S, D, V = plan.eval(_dev(w.sigma), _dev(w.mu), _dev(w.f_vol), None)
    torch.cuda.synchronize()
    ftrg = fjets.f_at_targets(w.volume, w.f_vol, w.tx, w.ty, w.inside, w.boundary, rows=1)
    So, Do, Vo = _oracle(w, alpha, plan.info()["delta"], ftrg)
    errs = [rel_err(S.cpu().numpy(), So), rel_err(D.cpu().numpy(), Do), rel_err(V.cpu().numpy(), Vo)]
    print(f"errors {errs}", flush=True)
    assert max(errs) < TOL


def test_order2_without_jets_config0():
    w = synth.config0()
    print("case order 2 eval without f_trg config0", flush=True)
    plan = _plan(w, 10.0, local_order=2)
    S, D, V = plan.eval(_dev(w.sigma), _dev(w.mu), _dev(w.f_vol), None)
    torch.cuda.synchronize()
    ftrg = fjets.f_at_targets(w.volume, w.f_vol, w.tx, w.ty, w.inside, w.boundary, rows=6)
    So, Do, Vo = _oracle(w, 10.0, plan.info()["delta"], ftrg, order=2)
    errs = [rel_err(S.cpu().numpy(), So), rel_err(D.cpu().numpy(), Do), rel_err(V.cpu().numpy(), Vo)]
    print(f"errors {errs}", flush=True)
    assert max(errs) < TOL


def test_multibody_without_f_trg_sampled():
    """3-body workload (cut cells with curved and sliver triangles) at
    alpha = 30: stratified sample against the oracle; the FP32 path at
    1e-6 with FP64 inputs."""
    w = small_multibody()
    alpha = 30.0
    print("case eval without f_trg multibody", flush=True)
    plan = _plan(w, alpha)
    S, D, V = [o.cpu().numpy().ravel() for o in plan.eval(_dev(w.sigma), _dev(w.mu), _dev(w.f_vol), None)]
    info = plan.info()
    sub = stratified_subset(w, info["band_volume"])
    ftrg = fjets.f_at_targets(w.volume, w.f_vol, w.tx, w.ty, w.inside, w.boundary, rows=1)
    So, Do, Vo = _oracle(w, alpha, info["delta"], ftrg, subset=sub)
    errs = [rel_err(S[sub], So), rel_err(D[sub], Do), rel_err(V[sub], Vo)]
    print(f"fp64 errors {errs}", flush=True)
    assert max(errs) < TOL
    import paper_2606_28865_amd as M
    p32 = _plan(w, alpha, tol=1e-6, prec=M.MHK_FP32, in64=1)
    S, D, V = [o.cpu().numpy().astype(np.float64).ravel()
               for o in p32.eval(_dev(w.sigma), _dev(w.mu), _dev(w.f_vol), None)]
    So, Do, Vo = _oracle(w, alpha, p32.info()["delta"], ftrg, subset=sub)
    errs = [rel_err(S[sub], So), rel_err(D[sub], Do), rel_err(V[sub], Vo)]
    print(f"fp32 errors {errs}", flush=True)
    assert max(errs) < 1e-6
