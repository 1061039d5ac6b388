"""Throughput of the kernel-split potential evaluation on one MI355X.

One step evaluates S[sigma], D[mu] and V[f] at every target of the
multi-body workload (10 seeded starfish bodies in [-1,1]^2, 16384 boundary
nodes, ~1.04M cut-cell volume nodes, 1M targets inside the bodies plus the
16384 boundary nodes), FP64, tolerance 1e-10, once for each alpha in
{1, 10, 100}; a target-eval is S, D and V at one target for one density.
Inputs and plans are resident in HBM before the timed region.

Prints one JSON line with throughput, the roofline of the dominant kernel
(measured with HIP events on the plan's stream inside the timed region) and
the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8000.0          # GB/s
FP64_PEAK = 78.6           # TFLOP/s, vector FP64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--alphas", type=str, default="1,10,100")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--cpu-sample", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {a.gpus}); the per-GPU "
              "throughput at N=1 is the figure this workload reports.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2606_28865_amd as M
    import synth

    t0 = time.time()
    w = synth.multibody()
    gen_s = time.time() - t0
    log(f"workload {w.name} generated in {gen_s:.1f} s")
    alphas = [float(x) for x in a.alphas.split(",")]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)
    sigma, mu, fv, ft = t(w.sigma), t(w.mu), t(w.f_vol), t(w.f_trg)
    plans, plan_s = [], []
    for al in alphas:
        t1 = time.time()
        prm = M.make_params(alpha=al, tol=a.tol, dx=w.dx)
        p = M.Plan(prm, w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True)
        torch.cuda.synchronize()
        plan_s.append(time.time() - t1)
        plans.append(p)
        log(f"plan alpha={al}: {plan_s[-1]:.1f} s, grid {p.info()['n_fine']}, {p.info()['device_bytes'] / 1e9:.2f} GB")
    n_out = plans[0].n_out
    outs = [p.eval(sigma, mu, fv, ft) for p in plans]
    for _ in range(a.warmup):
        for p, o in zip(plans, outs):
            p.eval(sigma, mu, fv, ft, out=o)
    torch.cuda.synchronize()
    log("warmup done")
    for p in plans:
        p.set_timing(True)
    stage = {k: [0.0] * len(plans) for k in ("ms_spread", "ms_fft", "ms_multiply", "ms_interp", "ms_levels",
                                             "ms_local", "ms_total")}
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    wall0 = time.perf_counter()
    for _ in range(a.steps):
        for i, (p, o) in enumerate(zip(plans, outs)):
            p.eval(sigma, mu, fv, ft, out=o)
            inf = p.info()
            for k in stage:
                stage[k][i] += inf[k]
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = ev0.elapsed_time(ev1)
    ms_step = ms / a.steps
    evals = n_out * len(plans)
    value = evals / (ms_step * 1e-3)
    for k in stage:
        stage[k] = [x / a.steps for x in stage[k]]
    infos = [p.info() for p in plans]

    # dominant kernel: the one with the largest summed time over the step
    tot = {k: sum(v) for k, v in stage.items() if k != "ms_total"}
    dom = max(tot, key=tot.get)
    roof = roofline(dom, stage, infos, w, plans)

    log(f"timed {a.steps} steps: {ms_step:.2f} ms/step")
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(w, infos, alphas, a.cpu_sample)

    line = {
        "metric": "target evals/s (S, D, V per target, FP64, rel err 1e-10 vs oracle)",
        "value": value,
        "unit": "target-evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "multibody-10-starfish", "n_boundary": w.n_b, "n_volume": w.n_v,
                   "n_targets": w.n_t, "n_out": n_out, "alphas": alphas, "tol": a.tol,
                   "batch": 1, "parallelism": "none"},
        "stage_ms": {k: [round(x, 4) for x in v] for k, v in stage.items()},
        "grid": [int(i["n_fine"]) for i in infos],
        "delta": [i["delta"] for i in infos],
        "plan_s": [round(x, 3) for x in plan_s],
        "gen_s": round(gen_s, 2),
        "wall_s": round(wall, 3),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def roofline(dom, stage, infos, w, plans):
    """Algorithmic bytes or flops of the dominant stage per launch over its
    measured HIP-event time."""
    name = dom[3:]
    if name == "levels":
        # pairs within the level radii, counted from the plan geometry on the host
        flops = 0.0
        for info in infos:
            flops += level_flops(w, info)
        t = sum(stage[dom]) * 1e-3
        ach = flops / t / 1e12
        return {"kernel": "k_level_sums", "bound": "alu", "achieved": ach, "peak": FP64_PEAK,
                "unit": "TFLOP/s", "frac": ach / FP64_PEAK, "traffic": None}
    if name in ("fft", "spread", "multiply", "interp"):
        byts = 0.0
        for info in infos:
            n = info["n_fine"]
            if n == 0:
                continue
            grid = n * (n + 2) * 8.0
            if name == "fft":
                byts += (4 + 4 + 3 + 3) * grid            # read + write per field, forward 4, inverse 3
            elif name == "multiply":
                nf = min(1.0, 1.0 / 2.0)
                byts += (4 + 3) * grid * 0.5 * 0 + (4 + 3) * grid * 0.5 + 0 * nf
            elif name == "spread":
                byts += 4 * grid + (w.n_v * 32 + w.n_b * 56)
            else:
                byts += 3 * grid + info["n_out"] * (16 + 24)
        t = sum(stage[dom]) * 1e-3
        ach = byts / t / 1e9
        return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK, "unit": "GB/s",
                "frac": ach / HBM_PEAK, "traffic": None}
    return {"kernel": name, "bound": "alu", "achieved": None, "peak": FP64_PEAK, "unit": "TFLOP/s",
            "frac": None, "traffic": None}


LEVEL_FLOPS_PER_PAIR = 64.0   # distance 5, compare 1, segment 4, 2 x 11 FMA table (44), S 2, D 4, misc 4


def level_flops(w, info):
    """Pairs (target, child node) with r < R_j summed over the levels, times
    the flops the level sum spends on one pair."""
    from scipy.spatial import cKDTree
    tg = np.concatenate([np.stack([w.tx, w.ty], 1), np.stack([w.boundary["x"], w.boundary["y"]], 1)])
    b = w.boundary
    pairs = 0
    for j in range(1, info["J"] + 1):
        R = info["level_radius"][j - 1]
        # child nodes: the level sum's sources lie on the same curves as the
        # panel nodes with 2^j times the density; count with the parent nodes
        tree = cKDTree(np.stack([b["x"], b["y"]], 1))
        cnt = tree.query_ball_point(tg, R, return_length=True)
        pairs += float(np.sum(cnt)) * (1 << j)
    return pairs * LEVEL_FLOPS_PER_PAIR


def cpu_baseline(w, infos, alphas, n_sample):
    """The oracle (plain direct sums, OpenMP) on n_sample targets of the same
    workload for alpha = alphas[len//2], scaled to target-evals/s."""
    import oracle as O
    i = len(alphas) // 2
    info = infos[i]
    g = np.random.default_rng(1)
    sub = np.sort(g.choice(w.n_t + w.n_b, n_sample, replace=False)).astype(np.int64)
    P = O.Problem(alphas[i], info["delta"], info["J"], w.boundary, volume=w.volume, targets=(w.tx, w.ty),
                  inside=w.inside, on_surface=True, sigma=w.sigma, mu=w.mu, f_vol=w.f_vol, f_trg=w.f_trg)
    t0 = time.perf_counter()
    P.eval(sub)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_sample / dt, "unit": "target-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_sample} random targets of the same workload at alpha={alphas[i]}, {dt:.1f} s"}


if __name__ == "__main__":
    main()
