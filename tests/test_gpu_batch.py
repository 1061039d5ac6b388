"""Batched evaluation and HIP-graph replay.

A plan with batch = b evaluates b densities per call; the whole evaluation
can be recorded once into a HIP graph bound to fixed buffers and replayed.
Every replay is compared with an eager evaluation of the same inputs, with
eager work and synchronisations between replays, and the input contents
changed between replays."""
import numpy as np
import pytest

import synth
from helpers import oracle_eval, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


@pytest.mark.parametrize("prec,geom", [(0, False), (1, False), (0, True)])
def test_graph_replay_matches_eager(prec, geom):
    """geom: the closest points recomputed inside the graph (MHK_PART_GEOMETRY)."""
    import paper_2606_28865_amd as M
    w = synth.config0()
    B = 5
    dt = torch.float64 if prec == 0 else torch.float32
    tol = 1e-10 if prec == 0 else 1e-6
    parts = M.PART_ALL | (M.PART_GEOMETRY if geom else 0)
    print(f"case graph replay prec={prec} batch={B} geometry={geom}", flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        prm = M.make_params(alpha=10.0, tol=tol, prec=prec, dx=w.dx, batch=B)
        plan = M.Plan(prm, w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True, stream=stream)
        eager = M.Plan(prm, w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True, stream=stream)
        sig = torch.zeros((B, w.n_b), dtype=dt, device="cuda")
        mu = torch.zeros_like(sig)
        fv = torch.zeros((B, w.n_v), dtype=dt, device="cuda")
        ft = torch.zeros((B, w.n_t + w.n_b), dtype=dt, device="cuda")
        out = plan.capture(sig, mu, fv, ft, parts=parts)
        g = np.random.default_rng(11)
        for rep in range(4):
            scale = g.uniform(0.5, 2.0, B)
            sig.copy_(_t(np.stack([w.sigma * s for s in scale]), dt))
            mu.copy_(_t(np.stack([w.mu * (1 + 0.1 * rep) for _ in scale]), dt))
            fv.copy_(_t(np.stack([w.f_vol * s for s in scale]), dt))
            ft.copy_(_t(np.stack([w.f_trg * s for s in scale]), dt))
            plan.replay()
            ref = eager.eval(sig, mu, fv, ft)
            stream.synchronize()
            for o, r in zip(out, ref):
                e = rel_err(o.cpu().numpy(), r.cpu().numpy())
                assert e < (1e-13 if prec == 0 else 1e-6), (rep, e)
            # unrelated eager work between replays
            x = torch.randn(1 << 20, device="cuda")
            (x * 2).sum().item()
    # the last replay against the oracle for one density
    k = 2
    So, Do, Vo = oracle_eval(w, 10.0, plan.info()["delta"], 3, sigma=sig[k].double().cpu().numpy(),
                             mu=mu[k].double().cpu().numpy(), f_vol=fv[k].double().cpu().numpy(),
                             f_trg=ft[k].double().cpu().numpy())
    lim = 1e-10 if prec == 0 else 1e-6
    assert rel_err(out[0][k].double().cpu().numpy(), So) < lim
    assert rel_err(out[1][k].double().cpu().numpy(), Do) < lim
    assert rel_err(out[2][k].double().cpu().numpy(), Vo) < lim


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_chunks_match_single(prec):
    """batch = 6 spans two chunks of the level kernel; each density equals its
    single evaluation (FP64: to 1e-13; FP32: to 1e-6)."""
    import paper_2606_28865_amd as M
    w = synth.config0()
    B = 6
    dt = torch.float64 if prec == 0 else torch.float32
    tol = 1e-10 if prec == 0 else 1e-6
    print(f"case batch chunks prec={prec}", flush=True)
    prm = M.make_params(alpha=10.0, tol=tol, prec=prec, dx=w.dx, batch=B)
    plan = M.Plan(prm, w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True)
    one = M.Plan(M.make_params(alpha=10.0, tol=tol, prec=prec, dx=w.dx), w.boundary, w.volume,
                 (w.tx, w.ty, w.inside), on_surface=True)
    g = np.random.default_rng(2)
    sig = np.stack([w.sigma + 0.1 * g.standard_normal(w.n_b) for _ in range(B)])
    mu = np.stack([w.mu * (k + 1) for k in range(B)])
    fv = np.stack([w.f_vol * (k - 2.5) for k in range(B)])
    ft = np.stack([w.f_trg * (k - 2.5) for k in range(B)])
    out = plan.eval(_t(sig, dt), _t(mu, dt), _t(fv, dt), _t(ft, dt))
    for k in range(B):
        ref = one.eval(_t(sig[k], dt), _t(mu[k], dt), _t(fv[k], dt), _t(ft[k], dt))
        torch.cuda.synchronize()
        for o, r in zip(out, ref):
            e = rel_err(o[k].double().cpu().numpy(), r.double().cpu().numpy())
            assert e < (1e-13 if prec == 0 else 1e-6), (k, e)


@pytest.mark.parametrize("prec", [0, 1])
def test_fewer_densities_than_the_batch(prec):
    """mhk_eval_batch: a plan sized for 6 densities evaluates 1, 3 and 6 of
    them (each stage over that many), equal to single-density evaluations;
    a full-batch graph captured afterwards still replays all 6."""
    import paper_2606_28865_amd as M
    w = synth.config0()
    B = 6
    dt = torch.float64 if prec == 0 else torch.float32
    tol = 1e-10 if prec == 0 else 1e-6
    lim = 1e-13 if prec == 0 else 1e-6
    g = np.random.default_rng(21)
    sig = np.stack([w.sigma * (1 + 0.1 * k) + 0.05 * g.standard_normal(w.n_b) for k in range(B)])
    mu = np.stack([w.mu * (1 - 0.1 * k) for k in range(B)])
    fv = np.stack([w.f_vol * (k + 1) for k in range(B)])
    ft = np.stack([w.f_trg * (k + 1) for k in range(B)])
    prm = lambda b: M.make_params(alpha=10.0, tol=tol, prec=prec, dx=w.dx, batch=b)
    plan = M.Plan(prm(B), w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True)
    single = M.Plan(prm(1), w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True)
    ref = [single.eval(_t(sig[k], dt), _t(mu[k], dt), _t(fv[k], dt), _t(ft[k], dt)) for k in range(B)]
    ref = [[o.cpu().numpy().ravel() for o in r] for r in ref]
    for nb in (1, 3, 6, 2):
        print(f"case nbatch={nb} of {B} prec={prec}", flush=True)
        out = plan.eval(_t(sig[:nb], dt), _t(mu[:nb], dt), _t(fv[:nb], dt), _t(ft[:nb], dt), nbatch=nb)
        torch.cuda.synchronize()
        assert out[0].shape == (nb, w.n_t + w.n_b)
        for k in range(nb):
            for o, r in zip(out, ref[k]):
                assert rel_err(o[k].cpu().numpy(), r) < lim, (nb, k, rel_err(o[k].cpu().numpy(), r))
    with pytest.raises(ValueError):
        plan.eval(_t(sig[:1], dt), _t(mu[:1], dt), _t(fv[:1], dt), _t(ft[:1], dt), nbatch=B + 1)
    # the library itself rejects a count beyond the plan's batch
    import ctypes as C
    x = _t(sig, dt)
    o = torch.empty((B, w.n_t + w.n_b), dtype=dt, device="cuda")
    rc = M.lib().mhk_eval_batch(plan._h, B + 1, M.PART_ALL, C.c_void_p(x.data_ptr()), None, None, None,
                                C.c_void_p(o.data_ptr()), None, None)
    assert rc == -1
    ins = (_t(sig, dt), _t(mu, dt), _t(fv, dt), _t(ft, dt))
    gout = plan.capture(*ins)
    plan.replay()
    torch.cuda.synchronize()
    for k in range(B):
        for o, r in zip(gout, ref[k]):
            assert rel_err(o[k].cpu().numpy(), r) < lim


def test_persistent_level_sums_graph_replay():
    """The persistent level-sum launch (its work counter zeroed by a kernel
    before each launch) inside a captured graph, replayed with new inputs,
    equals eager evaluations of a non-persistent plan."""
    import paper_2606_28865_amd as M
    w = synth.config0()
    B = 3
    print("case persistent level sums under graph replay", flush=True)
    mk = lambda ps: M.Plan(M.make_params(alpha=10.0, tol=1e-10, dx=w.dx, batch=B, lv_persist=ps), w.boundary,
                           w.volume, (w.tx, w.ty, w.inside), on_surface=True)
    plan, ref = mk(1), mk(0)
    sig = torch.zeros((B, w.n_b), dtype=torch.float64, device="cuda")
    mu = torch.zeros_like(sig)
    fv = torch.zeros((B, w.n_v), dtype=torch.float64, device="cuda")
    ft = torch.zeros((B, w.n_t + w.n_b), dtype=torch.float64, device="cuda")
    out = plan.capture(sig, mu, fv, ft)
    g = np.random.default_rng(5)
    for rep in range(3):
        sig.copy_(_t(np.stack([w.sigma * g.uniform(0.5, 1.5) for _ in range(B)])))
        mu.copy_(_t(np.stack([w.mu * g.uniform(0.5, 1.5) for _ in range(B)])))
        fv.copy_(_t(np.stack([w.f_vol * (k + 1) for k in range(B)])))
        ft.copy_(_t(np.stack([w.f_trg * (k + 1) for k in range(B)])))
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        e = ref.eval(sig, mu, fv, ft)
        torch.cuda.synchronize()
        for a, b in zip(out, e):
            assert rel_err(a.cpu().numpy(), b.cpu().numpy()) < 1e-13, rep
