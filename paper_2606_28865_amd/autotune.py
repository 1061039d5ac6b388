"""Autotuner for the history grid (oversampling factor, window width) and
the tile shapes of the dyadic-level sums (targets per workgroup, densities
per pass).

For one geometry, alpha, tolerance and precision, each candidate (upsamp,
wspread) is built as a plan with the same split delta, timed on the device
with HIP events over a few evaluations, and checked against a reference
evaluation by a more accurate plan (FP64, the tolerance / 1000, the default
grid) of the same inputs as the candidate sees them (for an FP32 candidate,
the densities rounded to FP32: the grid is tuned for the numerical error of
the evaluation, not for the rounding of its inputs, which the local layer
terms amplify through the density's second derivative): a candidate is
admissible when its relative max-norm difference to the reference is below
the tolerance for S, D and V.  The fastest admissible candidate wins.
Then, on that grid, the level-sum tile shapes (lv_block 256 or 512 targets
per workgroup; lv_bch 2, 4 or 8 densities per pass when batch > 1; one persistent launch per level or one wavefront
per work item) are timed the same way; they change only the order of the sums, so their results are
checked against the same reference and the fastest is kept.  Results are
cached in a JSON file keyed by the problem's sizes and parameters.

Everything runs through the library (no CPU fallback); the reference is the
library's own FP64 path, whose agreement with the oracle is what the parity
tests establish.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import _lib as L

DEFAULT_CANDIDATES = [(2.0, 0), (1.75, 0), (1.5, 0), (2.0, -1), (1.5, 1), (1.25, 2)]
CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mhk_autotune.json")


def _key(geometry, alpha, tol, prec, batch, tiles=True):
    b, v, t = geometry["boundary"], geometry.get("volume"), geometry["targets"]
    return (f"nb{len(b['x'])}-nv{0 if v is None else len(v['x'])}-nt{len(t[0])}-a{alpha:g}-t{tol:g}-p{prec}"
            f"-b{batch}" + ("-tiles" if tiles else ""))


def _rel(a, b):
    a = a.double().cpu().numpy().ravel()
    b = b.double().cpu().numpy().ravel()
    m = np.isfinite(b)
    s = np.abs(b[m]).max()
    return float(np.abs(a[m] - b[m]).max() / (s if s > 0 else 1.0))


def tile_candidates(batch):
    """(lv_block, lv_bch, lv_persist) triples tried on the chosen grid."""
    bchs = (1,) if batch == 1 else tuple(b for b in (2, 4, 8) if b <= max(2, batch))
    return [(nb, bc, ps) for ps in (0, 1) for nb in (256, 512) for bc in bchs]


def tune(geometry, alpha, tol, prec, densities, dx=0.0, delta=0.0, batch=1, candidates=None, reps=3,
         cache=CACHE, log=None, tiles=True):
    """geometry: dict(boundary=..., volume=..., targets=(x, y, inside), on_surface=bool);
    densities: (sigma, mu, f_vol, f_trg) host arrays of one density.
    Returns dict(upsamp, wspread, ms, err, table)."""
    import torch
    key = _key(geometry, alpha, tol, prec, batch, tiles)
    if cache and os.path.exists(cache):
        try:
            db = json.load(open(cache))
            if key in db:
                return db[key]
        except (OSError, ValueError):
            pass
    cands = candidates or DEFAULT_CANDIDATES
    if delta <= 0:
        delta = L.resolve_params(alpha=alpha, tol=tol, prec=prec, dx=dx)["delta"]
    geo = (geometry["boundary"], geometry.get("volume"), geometry["targets"])
    on = geometry.get("on_surface", True)
    dt = torch.float64 if prec == L.MHK_FP64 else torch.float32

    def dev(a, d):
        a = np.ascontiguousarray(a)
        a = np.broadcast_to(a, (batch,) + a.shape).copy()
        return torch.as_tensor(a, dtype=d, device="cuda")

    ref_plan = L.Plan(L.make_params(alpha=alpha, tol=max(1e-13, tol * 1e-3), delta=delta, batch=1), *geo,
                      on_surface=on)
    ref = ref_plan.eval(*(dev(x, dt)[:1].to(torch.float64) for x in densities))
    torch.cuda.synchronize()
    ref_plan.close()
    ins = [dev(x, dt) for x in densities]
    w0 = L.resolve_params(alpha=alpha, tol=tol, prec=prec, delta=delta)["wspread"]
    def trial(ups, ws, lv_block=0, lv_bch=0, lv_persist=0):
        try:
            p = L.Plan(L.make_params(alpha=alpha, tol=tol, prec=prec, delta=delta, batch=batch, upsamp=ups,
                                     wspread=ws, lv_block=lv_block, lv_bch=lv_bch, lv_persist=lv_persist), *geo,
                       on_surface=on)
        except L.MhkError as e:
            return {"upsamp": ups, "wspread": ws, "lv_block": lv_block, "lv_bch": lv_bch, "lv_persist": lv_persist,
                    "error": str(e)}
        out = p.eval(*ins)
        torch.cuda.synchronize()
        err = max(_rel(o[0], r[0]) for o, r in zip(out, ref))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            p.eval(*ins, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        info = p.info()
        p.close()
        del out
        if log:
            log(f"autotune alpha={alpha} ups={ups} w={ws} lv_block={lv_block} lv_bch={lv_bch} "
                f"lv_persist={lv_persist}: {ms:.3f} ms, err {err:.2e}, n {info['n_fine']}")
        return {"upsamp": ups, "wspread": ws, "lv_block": lv_block, "lv_bch": lv_bch, "lv_persist": lv_persist,
                "ms": ms, "err": err, "n_fine": info["n_fine"]}

    table = [trial(ups, max(4, min(16, w0 + dw))) for ups, dw in cands]
    ok = [c for c in table if "ms" in c and c["err"] < tol]
    if not ok:
        raise RuntimeError(f"autotune: no admissible candidate for {key}: {table}")
    best = min(ok, key=lambda c: c["ms"])
    tile_table = []
    if tiles:
        tile_table = [trial(best["upsamp"], best["wspread"], nb, bc, ps) for nb, bc, ps in tile_candidates(batch)]
        ok2 = [c for c in tile_table if "ms" in c and c["err"] < tol]
        if ok2:
            best = min(ok2 + [best], key=lambda c: c["ms"])
    res = {"upsamp": best["upsamp"], "wspread": best["wspread"], "lv_block": best["lv_block"],
           "lv_bch": best["lv_bch"], "lv_persist": best["lv_persist"], "ms": best["ms"], "err": best["err"],
           "table": table,
           "tile_table": tile_table, "delta": delta}
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            db = json.load(open(cache)) if os.path.exists(cache) else {}
            db[key] = res
            json.dump(db, open(cache, "w"), indent=1)
        except (OSError, ValueError):
            pass
    return res
