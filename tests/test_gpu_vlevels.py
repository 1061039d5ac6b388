"""Dyadic levels of the volume potential (v_levels = 1) against the
oracle (oracle/vlevels.py): V = V_H(delta) + sum_j V_j + V_L(delta*), FP64
at 1e-10 relative on a stratified sample of config 0's outputs; S and D are
those of a plan without volume levels; and V moves by no more than the
local expansion's own error when its time split moves from delta to
delta*."""
import numpy as np
import pytest

import synth
from helpers import oracle_eval, rel_err, stratified_subset
from oracle import vlevels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("alpha", [10.0, 3.0])
def test_volume_levels_config0(alpha):
    import paper_2606_28865_amd as M
    w = synth.config0()
    print(f"case volume levels config0 alpha={alpha}", flush=True)
    mk = lambda vl: M.Plan(M.make_params(alpha=alpha, tol=TOL, dx=w.dx, v_levels=vl), w.boundary, w.volume,
                           (w.tx, w.ty, w.inside), on_surface=True)
    plan = mk(1)
    info = plan.info()
    assert info["band_volume"] < mk(0).info()["band_volume"]
    S, D, V = [o.cpu().numpy().ravel() for o in plan.eval(_dev(w.sigma), _dev(w.mu), _dev(w.f_vol), _dev(w.f_trg))]
    torch.cuda.synchronize()
    sub = stratified_subset(w, info["band_layer"] * 8, n_each=48, seed=4)
    Vo = vlevels.volume_potential(w, alpha, info["delta"], info["J"], w.volume["rule"], w.f_trg, subset=sub)
    ev = rel_err(V[sub], Vo)
    So, Do, _ = oracle_eval(w, alpha, info["delta"], 3, subset=sub)
    es, ed = rel_err(S[sub], So), rel_err(D[sub], Do)
    # the plan without volume levels: V differs by the local expansion's error only
    p0 = mk(0)
    V0 = p0.eval(_dev(w.sigma), _dev(w.mu), _dev(w.f_vol), _dev(w.f_trg))[2].cpu().numpy().ravel()
    dv = np.abs(V - V0).max() / np.abs(V0).max()
    print(f"volume levels alpha={alpha}: V {ev:.2e} S {es:.2e} D {ed:.2e}; moved {dv:.2e} from the plain plan",
          flush=True)
    assert ev < TOL and es < TOL and ed < TOL
    assert dv > 0


def test_volume_levels_disk_closed_form():
    """V[1] in a disk of radius 0.5, (1 - alpha R K1(alpha R) I0(alpha r))/alpha^2
    inside: with the volume levels the local part's time split drops from
    delta to delta/64, and the error at the boundary nodes and the targets
    inside falls with it."""
    from scipy.special import i0, k1
    import paper_2606_28865_amd as M
    R, alpha = 0.5, 10.0
    cv = synth.Curve(r0=R)
    bnd = synth.discretize([cv], 24)
    vol = synth.cut_cell_volume([cv], 0.05)
    g = np.random.default_rng(3)
    rr = R * np.sqrt(g.uniform(size=400)); th = g.uniform(0, 2 * np.pi, 400)
    tx, ty = rr * np.cos(th), rr * np.sin(th)
    inside = np.ones(len(tx), np.int8)
    X = np.concatenate([tx, bnd["x"]]); Y = np.concatenate([ty, bnd["y"]])
    r = np.hypot(X, Y)
    exact = (1 - alpha * R * k1(alpha * R) * i0(alpha * r)) / alpha ** 2
    errs = {}
    for vl in (0, 1):
        plan = M.Plan(M.make_params(alpha=alpha, tol=1e-10, delta=2e-3, v_levels=vl), bnd, vol, (tx, ty, inside),
                      on_surface=True)
        V = plan.eval(None, None, _dev(np.ones(len(vol["x"]))), _dev(np.ones(len(X))))[2].cpu().numpy().ravel()
        errs[vl] = (np.abs(V[:len(tx)] - exact[:len(tx)]).max() / np.abs(exact).max(),
                    np.abs(V[len(tx):] - exact[len(tx):]).max() / np.abs(exact).max())
        plan.close()
    print(f"disk V[1] errors (targets, boundary nodes): plain {errs[0]}, volume levels {errs[1]}", flush=True)
    assert errs[1][0] < errs[0][0] and errs[1][1] < errs[0][1]


def test_volume_levels_fp32_fp64_inputs():
    """An FP32 plan (FP64 inputs) with volume levels against the FP64 oracle
    with volume levels: the FP32 level sums over the volume level nodes,
    within the FP32 bar of 1e-6."""
    import paper_2606_28865_amd as M
    w = synth.config0()
    alpha = 10.0
    print("case volume levels fp32 config0", flush=True)
    plan = M.Plan(M.make_params(alpha=alpha, tol=1e-6, prec=M.MHK_FP32, in64=1, dx=w.dx, v_levels=1), w.boundary,
                  w.volume, (w.tx, w.ty, w.inside), on_surface=True)
    info = plan.info()
    V = plan.eval(None, None, _dev(w.f_vol), _dev(w.f_trg))[2].cpu().numpy().astype(np.float64).ravel()
    torch.cuda.synchronize()
    sub = stratified_subset(w, info["band_layer"] * 8, n_each=48, seed=4)
    Vo = vlevels.volume_potential(w, alpha, info["delta"], info["J"], w.volume["rule"], w.f_trg, subset=sub)
    ev = rel_err(V[sub], Vo)
    print(f"volume levels fp32: V {ev:.2e}", flush=True)
    assert ev < 1e-6


def test_volume_levels_second_order():
    """A second-order plan with volume levels against the oracle at the same
    order (f's gradient and Hessian from the analytic sources), FP64 at
    1e-10."""
    import paper_2606_28865_amd as M
    w = synth.config0()
    alpha = 10.0
    X = np.concatenate([w.tx, w.boundary["x"]])
    Y = np.concatenate([w.ty, w.boundary["y"]])
    jet = w.meta["fsrc"].jet(X, Y)
    print("case volume levels order 2 config0", flush=True)
    plan = M.Plan(M.make_params(alpha=alpha, tol=TOL, dx=w.dx, v_levels=1, local_order=2), w.boundary, w.volume,
                  (w.tx, w.ty, w.inside), on_surface=True)
    info = plan.info()
    V = plan.eval(None, None, _dev(w.f_vol), _dev(jet))[2].cpu().numpy().ravel()
    torch.cuda.synchronize()
    sub = stratified_subset(w, info["band_layer"] * 8, n_each=48, seed=4)
    Vo = vlevels.volume_potential(w, alpha, info["delta"], info["J"], w.volume["rule"], jet[0], subset=sub,
                                  order=2, f_jet=jet[1:])
    ev = rel_err(V[sub], Vo)
    print(f"volume levels order 2: V {ev:.2e}", flush=True)
    assert ev < TOL


def test_volume_levels_without_f_trg():
    """Volume levels with f at the targets reconstructed by the plan (f_trg
    omitted) against the oracle fed the oracle's reconstruction."""
    import paper_2606_28865_amd as M
    from oracle import fjets
    w = synth.config0()
    alpha = 10.0
    print("case volume levels without f_trg config0", flush=True)
    plan = M.Plan(M.make_params(alpha=alpha, tol=TOL, dx=w.dx, v_levels=1), w.boundary, w.volume,
                  (w.tx, w.ty, w.inside), on_surface=True)
    info = plan.info()
    V = plan.eval(None, None, _dev(w.f_vol), None)[2].cpu().numpy().ravel()
    torch.cuda.synchronize()
    ftrg = fjets.f_at_targets(w.volume, w.f_vol, w.tx, w.ty, w.inside, w.boundary, rows=1)[0]
    sub = stratified_subset(w, info["band_layer"] * 8, n_each=48, seed=4)
    Vo = vlevels.volume_potential(w, alpha, info["delta"], info["J"], w.volume["rule"], ftrg, subset=sub)
    ev = rel_err(V[sub], Vo)
    print(f"volume levels without f_trg: V {ev:.2e}", flush=True)
    assert ev < TOL


def test_volume_levels_batch_matches_single():
    """A batch of three sources through the volume levels equals each source
    evaluated alone (FP64, 1e-13)."""
    import paper_2606_28865_amd as M
    w = synth.config0()
    alpha = 10.0
    B = 3
    scale = np.array([1.0, -0.5, 2.0])
    print("case volume levels batch 3 config0", flush=True)
    pb = M.Plan(M.make_params(alpha=alpha, tol=TOL, dx=w.dx, v_levels=1, batch=B), w.boundary, w.volume,
                (w.tx, w.ty, w.inside), on_surface=True)
    p1 = M.Plan(M.make_params(alpha=alpha, tol=TOL, dx=w.dx, v_levels=1), w.boundary, w.volume,
                (w.tx, w.ty, w.inside), on_surface=True)
    fv = np.stack([w.f_vol * s for s in scale])
    ft = np.stack([w.f_trg * s for s in scale])
    Vb = pb.eval(None, None, _dev(fv), _dev(ft))[2].cpu().numpy()
    for k in range(B):
        V1 = p1.eval(None, None, _dev(fv[k]), _dev(ft[k]))[2].cpu().numpy().ravel()
        e = rel_err(Vb[k], V1)
        print(f"density {k}: {e:.2e}", flush=True)
        assert e < 1e-13
