"""The request server on the GPU: requests of several plans (geometries,
alpha, tolerances, precisions) submitted together overlap on the device; each
result equals the same request evaluated alone, within the request's
tolerance, and agrees with the oracle; coalesced requests equal single ones;
heat-step chains equal the same steps taken directly; and a plan's
creation, use and destruction do not wait for other streams' work."""
import numpy as np
import pytest

import synth
from helpers import oracle_eval, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sims():
    from paper_2606_28865_amd.serve import Geometry
    out = []
    for si, (nb, nv, alpha, tol) in enumerate([(1024, 20000, 10.0, 1e-10), (2048, 40000, 3.0, 1e-6),
                                               (1024, 10000, 100.0, 1e-10)]):
        w = synth.multibody(cfg=200 + si, n_bodies=3, n_boundary=nb, n_volume=nv, n_targets=3000, box=0.6)
        out.append((w, Geometry(f"g{si}", w.boundary, w.volume, (w.tx, w.ty, w.inside), True), alpha, tol))
    return out


def test_mix_equals_alone():
    from paper_2606_28865_amd.serve import Request, Server
    sims = _sims()
    g = np.random.default_rng(0)

    def req(rid, si):
        w, geo, alpha, tol = sims[si]
        s = 1.0 + 0.2 * g.standard_normal()
        return Request(rid, geo, alpha, tol, 1 if tol >= 1e-6 else 0, w.sigma * s, w.mu * (2 - s), w.f_vol * s,
                       w.f_trg * s, dx=w.dx)

    print("case serve mix", flush=True)
    reqs = [req(i, i % 3) for i in range(12)]
    srv = Server(budget_bytes=8 << 30, max_inflight=6)
    for r in reqs:
        srv.submit(r)
    while srv.queue or srv.inflight:
        srv.step()
    assert len(srv.finished) == 12 and not srv.rejected
    # each request again, alone
    for r in reqs:
        again = Request(1000 + r.rid, r.geometry, r.alpha, r.tol, r.prec, r.sigma, r.mu, r.f_vol, r.f_trg, dx=r.dx)
        srv.submit(again)
        while srv.queue or srv.inflight:
            srv.step()
        lim = 1e-13 if r.prec == 0 else 1e-6
        for a, b in zip(r.result, again.result):
            assert rel_err(a, b) < lim, (r.rid, rel_err(a, b))
    # one request of each simulation against the oracle
    for si in range(3):
        r = reqs[si]
        w = sims[si][0]
        plan = srv.plans[r.plan_key]["plan"]
        sub = np.arange(0, w.n_t + w.n_b, 97, dtype=np.int64)
        ref = oracle_eval(w, r.alpha, plan.info()["delta"], 3, subset=sub,
                          sigma=np.asarray(r.sigma, np.float32 if r.prec else np.float64).astype(np.float64),
                          mu=np.asarray(r.mu, np.float32 if r.prec else np.float64).astype(np.float64),
                          f_vol=np.asarray(r.f_vol, np.float32 if r.prec else np.float64).astype(np.float64),
                          f_trg=np.asarray(r.f_trg, np.float32 if r.prec else np.float64).astype(np.float64))
        lim = 1e-10 if r.prec == 0 else 1e-6
        for a, b in zip(r.result, ref):
            assert rel_err(np.asarray(a, np.float64).ravel()[sub], b) < lim
    srv.close()


def test_coalesced_equals_alone():
    """Requests of one plan queued together are evaluated as one batch (the
    plan's batch dimension); each result equals the request evaluated alone
    on a plan without batching."""
    from paper_2606_28865_amd.serve import Request, Server
    sims = _sims()[:2]
    g = np.random.default_rng(1)

    def req(rid, si):
        w, geo, alpha, tol = sims[si]
        s = 1.0 + 0.2 * g.standard_normal()
        return Request(rid, geo, alpha, tol, 1 if tol >= 1e-6 else 0, w.sigma * s, w.mu * (2 - s), w.f_vol * s,
                       w.f_trg * s, dx=w.dx)

    print("case serve coalesced", flush=True)
    reqs = [req(i, i % 2) for i in range(8)]
    srv = Server(budget_bytes=8 << 30, max_inflight=6, max_batch=4)
    for r in reqs:
        srv.submit(r)
    while srv.queue or srv.inflight:
        srv.step()
    assert len(srv.finished) == 8 and not srv.rejected
    assert max(r.batched_with for r in reqs) == 4
    srv.close()
    alone = Server(budget_bytes=8 << 30, max_inflight=6, max_batch=1)
    for r in reqs:
        again = Request(1000 + r.rid, r.geometry, r.alpha, r.tol, r.prec, r.sigma, r.mu, r.f_vol, r.f_trg, dx=r.dx)
        alone.submit(again)
        while alone.queue or alone.inflight:
            alone.step()
        assert again.batched_with == 1
        lim = 1e-12 if r.prec == 0 else 1e-6
        for a, b in zip(r.result, again.result):
            assert rel_err(a, b) < lim, (r.rid, rel_err(a, b))
    alone.close()


def _heat_geometry(cfg, nb, nv):
    from paper_2606_28865_amd.serve import Geometry
    w = synth.multibody(cfg=cfg, n_bodies=3, n_boundary=nb, n_volume=nv, n_targets=10, box=0.6)
    vol = w.volume
    return w, Geometry(f"heat{cfg}", w.boundary, vol, (vol["x"], vol["y"], np.ones(len(vol["x"]), np.int8)), True)


def test_heat_chains_through_server():
    """Two heat-step chains (each step's input is the previous step's
    result, kept on the device) of different geometries and alpha run
    through the server beside eval requests; each chain ends where the same
    steps taken one after another directly end, and near the closed form
    c^n u0 of the sine mode."""
    import paper_2606_28865_amd as M
    from paper_2606_28865_amd.serve import HeatChain, Request, Server
    k = np.pi
    chains, ref = [], []
    for i, (cfg, nb, nv, alpha) in enumerate([(220, 1024, 20000, 10.0), (221, 2048, 30000, 4.0)]):
        w, geo = _heat_geometry(cfg, nb, nv)
        X = np.concatenate([w.volume["x"], w.boundary["x"]])
        Y = np.concatenate([w.volume["y"], w.boundary["y"]])
        u0 = np.sin(k * (X + 0.3)) * np.sin(k * (Y + 0.2))
        c = alpha ** 2 / (alpha ** 2 + 2 * k * k)
        gb = u0[len(w.volume["x"]):]
        chains.append(HeatChain(i, geo, alpha, 1e-10, u0, lambda n, gb=gb, c=c: c ** n * gb, 3, dx=w.dx,
                                rid0=100 * (i + 1)))
        ref.append((w, alpha, u0, gb, c))
    sims = _sims()
    g = np.random.default_rng(2)
    evals = []
    for i in range(4):
        w, geo, alpha, tol = sims[i % 3]
        s = 1.0 + 0.2 * g.standard_normal()
        evals.append(Request(i, geo, alpha, tol, 1 if tol >= 1e-6 else 0, w.sigma * s, w.mu, w.f_vol, w.f_trg,
                             dx=w.dx))
    print("case serve heat chains", flush=True)
    srv = Server(budget_bytes=16 << 30, max_inflight=6)
    for c in chains:
        srv.submit(c.first())
    for r in evals:
        srv.submit(r)
    while srv.queue or srv.inflight:
        srv.step()
    assert not srv.rejected, [r.error for r in srv.rejected]
    assert all(c.finished for c in chains)
    assert all(r.result is not None for r in evals)
    for c, (w, alpha, u0, gb, cc) in zip(chains, ref):
        got = c.steps[-1].result[0].cpu().numpy()
        plan = M.Plan(M.make_params(alpha=alpha, tol=1e-10, dx=w.dx), w.boundary, w.volume,
                      (w.volume["x"], w.volume["y"], np.ones(len(w.volume["x"]), np.int8)), on_surface=True)
        nys = M.Nystrom(alpha, w.boundary)
        u = torch.as_tensor(u0, dtype=torch.float64, device="cuda")
        for n in range(1, 4):
            u, _, _ = M.heat_step(plan, nys, u, torch.as_tensor(cc ** n * gb, dtype=torch.float64, device="cuda"),
                                  tol=1e-12)
        direct = u.cpu().numpy()
        assert rel_err(got, direct) < 1e-12, rel_err(got, direct)
        ex = cc ** 3 * u0
        # the split's own error at this coarse mesh (delta from dx): about 1e-3
        assert np.abs(got - ex).max() / np.abs(ex).max() < 5e-3
        plan.close()
        nys.close()
    srv.close()


def test_plan_lifecycle_keeps_other_work_running():
    """Creating, using and destroying a plan and a Nystrom object wait only
    for their own stream: evaluations queued on another plan's stream are
    still running after each of these steps.  Run in a child process: there
    the two streams get distinct hardware queues (HIP multiplexes streams
    onto a few hardware queues per process, and the hardware runs the work
    of streams sharing one in order, which no library call can avoid)."""
    import json
    import os
    import subprocess
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    print("case plan lifecycle beside queued evals (child process)", flush=True)
    r = subprocess.run([sys.executable, os.path.join(here, "lifecycle_child.py")], capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print(res, flush=True)
    assert all(res["pending"].values()), res
    assert res["finite"] and res["converged"]
