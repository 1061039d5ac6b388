"""Child process of test_gpu_serve.test_plan_lifecycle_keeps_other_work_running
(not collected): in a fresh process the first streams map to distinct
hardware queues, so the check sees the library's own waits only.  Prints
one JSON line."""
import json
import os
import sys
import time

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import paper_2606_28865_amd as M  # noqa: E402
import synth  # noqa: E402


def main():
    w = synth.multibody(cfg=230, n_bodies=5, n_boundary=8192, n_volume=400_000, n_targets=400_000)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    s1 = torch.cuda.Stream()
    with torch.cuda.stream(s1):
        big = M.Plan(M.make_params(alpha=10.0, tol=1e-10, dx=w.dx), w.boundary, w.volume, (w.tx, w.ty, w.inside),
                     on_surface=True, stream=s1)
        ins = (dev(w.sigma), dev(w.mu), dev(w.f_vol), dev(w.f_trg))
        out = big.eval(*ins)
        s1.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s1)
        for _ in range(3):
            big.eval(*ins, out=out)
        e1.record(s1)
        s1.synchronize()
        per = e0.elapsed_time(e1) / 3 / 1e3
        n = int(min(600, max(20, 0.7 / per)))
        for _ in range(n):
            big.eval(*ins, out=out)
        ev = torch.cuda.Event()
        ev.record(s1)
    w2 = synth.config0(n_panels=16, dx=0.2, grid=16)
    s2 = torch.cuda.Stream()
    pending = {}
    t0 = time.perf_counter()
    with torch.cuda.stream(s2):
        small = M.Plan(M.make_params(alpha=10.0, tol=1e-10, dx=w2.dx), w2.boundary, w2.volume,
                       (w2.tx, w2.ty, w2.inside), on_surface=True, stream=s2)
        pending["plan created"] = not ev.query()
        nys = M.Nystrom(10.0, w2.boundary, stream=s2)
        pending["Nystrom created"] = not ev.query()
        S, D, V = small.eval(dev(w2.sigma), dev(w2.mu), dev(w2.f_vol), dev(w2.f_trg))
        g = dev(np.cos(np.arange(w2.n_b)))
        mu_, u_, info = M.solve_dirichlet(small, nys, g, dev(w2.f_vol), dev(w2.f_trg), tol=1e-12)
        s2.synchronize()
        pending["evaluated and solved"] = not ev.query()
        Sh = S.cpu().numpy()
        phases = small.info()["ms_plan"]
        small.close()
        nys.close()
        pending["destroyed"] = not ev.query()
    ms = (time.perf_counter() - t0) * 1e3
    s1.synchronize()
    big.close()
    print(json.dumps({"queued_evals": n, "ms_per_eval": per * 1e3, "ms": ms, "pending": pending,
                      "plan_phases_ms": phases, "finite": bool(np.isfinite(Sh).all()),
                      "converged": bool(info["converged"])}), flush=True)


if __name__ == "__main__":
    main()
