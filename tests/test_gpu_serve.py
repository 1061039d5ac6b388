"""The request server on the GPU: requests of several plans (geometries,
alpha, tolerances, precisions) submitted together overlap on the device; each
result equals the same request evaluated alone, within the request's
tolerance, and agrees with the oracle."""
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
