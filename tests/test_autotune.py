"""Grid autotuner: the cache and its key on the CPU; on the device, the
chosen candidate is admissible, is the fastest admissible one of its table,
and a plan built with it agrees with the oracle to the requested tolerance."""
import json

import numpy as np
import pytest

import synth
from helpers import oracle_eval, rel_err


def _geometry(w):
    return {"boundary": w.boundary, "volume": w.volume, "targets": (w.tx, w.ty, w.inside), "on_surface": True}


def test_cache_key_and_hit(tmp_path):
    pytest.importorskip("torch")
    from paper_2606_28865_amd import autotune
    w = synth.config0()
    geo = _geometry(w)
    k1 = autotune._key(geo, 10.0, 1e-6, 1, 1)
    # every tuned quantity is part of the key
    assert len({k1, autotune._key(geo, 10.0, 1e-6, 1, 64), autotune._key(geo, 3.0, 1e-6, 1, 1),
                autotune._key(geo, 10.0, 1e-10, 1, 1), autotune._key(geo, 10.0, 1e-6, 0, 1),
                autotune._key(geo, 10.0, 1e-6, 1, 1, tiles=False)}) == 6
    # tile shapes tried on the chosen grid: densities per pass only with a batch
    assert autotune.tile_candidates(1) == [(n, 1, p) for p in (0, 1) for n in (256, 512)]
    assert autotune.tile_candidates(64) == [(n, b, p) for p in (0, 1) for n in (256, 512) for b in (2, 4, 8)]
    entry = {"upsamp": 1.5, "wspread": 9, "ms": 1.0, "err": 1e-7, "table": [], "delta": 1e-3}
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({k1: entry}))
    # a cached entry is returned as stored, without building a plan
    got = autotune.tune(geo, 10.0, 1e-6, 1, (w.sigma, w.mu, w.f_vol, w.f_trg), dx=w.dx, batch=1,
                        cache=str(cache))
    assert got == entry


@pytest.mark.gpu
def test_tuned_plan_matches_oracle():
    torch = pytest.importorskip("torch")
    import paper_2606_28865_amd as M
    from paper_2606_28865_amd import autotune
    w = synth.config0()
    alpha, tol = 10.0, 1e-6
    print("case autotune config0 fp32 batch 2", flush=True)
    res = autotune.tune(_geometry(w), alpha, tol, M.MHK_FP32, (w.sigma, w.mu, w.f_vol, w.f_trg), dx=w.dx,
                        batch=2, candidates=[(2.0, 0), (1.5, 1), (1.25, 2)], reps=2, cache=None)
    ok = [c for c in res["table"] + res["tile_table"] if "ms" in c and c["err"] < tol]
    assert ok and res["err"] < tol
    assert res["ms"] == min(c["ms"] for c in ok)
    assert len(res["tile_table"]) == 4
    prm = M.make_params(alpha=alpha, tol=tol, prec=M.MHK_FP32, delta=res["delta"], upsamp=res["upsamp"],
                        wspread=res["wspread"], lv_block=res["lv_block"], lv_bch=res["lv_bch"],
                        lv_persist=res["lv_persist"])
    plan = M.Plan(prm, w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True)
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    out = plan.eval(f32(w.sigma), f32(w.mu), f32(w.f_vol), f32(w.f_trg))
    torch.cuda.synchronize()
    r = lambda a: np.asarray(a, np.float32).astype(np.float64)
    ref = oracle_eval(w, alpha, plan.info()["delta"], 3, sigma=r(w.sigma), mu=r(w.mu), f_vol=r(w.f_vol),
                      f_trg=r(w.f_trg))
    errs = [rel_err(o.cpu().numpy().astype(np.float64), e) for o, e in zip(out, ref)]
    print(f"autotune pick ups {res['upsamp']} w {res['wspread']}: errs {errs}", flush=True)
    assert max(errs) < tol
