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
FP32_PEAK = 157.3
FP64_PEAK = 78.6           # TFLOP/s, vector FP64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--alphas", type=str, default="1,10,100")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--check-each", type=int, default=8,
                    help="outputs per stratum and alpha of the parity check against the oracle")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the parity check and the CPU baseline (profiling runs only)")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32 half of the metric (its 4M-target workload)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB device-to-device 4 times (calibrates HBM byte counters)")
    ap.add_argument("--workload", default="multibody",
                    choices=["multibody", "precision", "batched", "serve", "bie", "heat"],
                    help="multibody: the default throughput line; precision: FP32 vs FP64 at tol 1e-6 on "
                         "64k boundary / 4M volume / 4M targets; batched: 64 densities per call under a "
                         "captured HIP graph; serve: Poisson stream of Rothe-step requests; bie: Dirichlet "
                         "solve (Nystrom matrix, GMRES) on the 10-body geometry; heat: implicit-Euler "
                         "heat steps with the volume nodes as targets")
    ap.add_argument("--order", type=str, default="",
                    help="order in which a step enqueues the alpha plans, e.g. 0,1,2 (default: reversed)")
    ap.add_argument("--one-stream", action="store_true",
                    help="evaluate the three alpha plans one after another on one stream (default: each plan "
                         "on its own stream, the three evaluations of a step concurrent)")
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--requests", type=int, default=120)
    ap.add_argument("--max-batch", type=int, default=4,
                    help="serve: requests of one plan coalesced into one launch")
    ap.add_argument("--heat-steps", type=int, default=8, help="serve: steps of each heat chain")
    ap.add_argument("--lv-block", type=int, default=0, help="level-sum workgroup size (0: the plan's default)")
    ap.add_argument("--lv-persist", type=int, default=0, help="1: persistent level-sum launch")
    ap.add_argument("--no-per-potential", action="store_true",
                    help="skip the per-potential rates (profiling runs: only the step's own launches)")
    return ap.parse_args()


def copy_probe():
    """A plain device copy of known size: 256 MiB read + 256 MiB written per
    dispatch; the FETCH_SIZE / WRITE_SIZE counters of this dispatch give the
    scale factor of the counters on this GPU."""
    import torch
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": a.numel() * 8, "dispatches": 4}), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.copy_probe:
        copy_probe()
        return
    if a.gpus != 1:
        print(f"bench.py: the library runs on one GPU (got --gpus {a.gpus}); the reported "
              "figure is one GPU's throughput, at N=1.", file=sys.stderr)
        sys.exit(2)
    if a.workload != "multibody":
        {"precision": run_precision, "batched": run_batched, "serve": run_serve, "bie": run_bie,
         "heat": run_heat}[a.workload](a)
        return
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
    # The three alpha problems of a step are independent: by default each plan
    # has its own stream (default priority), the step forks them from the
    # caller's stream and joins them back, so one plan's tail overlaps the
    # next plan's start.
    cur = torch.cuda.current_stream()
    streams = [cur] * len(alphas) if a.one_stream else [torch.cuda.Stream() for _ in alphas]
    plans, plan_s = [], []
    for al, s in zip(alphas, streams):
        t1 = time.time()
        prm = M.make_params(alpha=al, tol=a.tol, dx=w.dx, lv_block=a.lv_block, lv_persist=a.lv_persist)
        p = M.Plan(prm, w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True, stream=s)
        torch.cuda.synchronize()
        plan_s.append(time.time() - t1)
        plans.append(p)
        log(f"plan alpha={al}: {plan_s[-1]:.1f} s, grid {p.info()['n_fine']}, {p.info()['device_bytes'] / 1e9:.2f} GB")
    n_out = plans[0].n_out
    # One step = the whole hot path for every plan, the closest-point search
    # and local coefficients of every target included (MHK_PART_GEOMETRY);
    # the rate with the geometry kept from plan creation is reported beside.
    fresh = M.PART_ALL | M.PART_GEOMETRY
    outs = []
    for p, s in zip(plans, streams):
        with torch.cuda.stream(s):
            outs.append(p.eval(sigma, mu, fv, ft, parts=fresh))
    torch.cuda.synchronize()

    # order in which a step enqueues the plans (indices into alphas): with
    # the plans on their own streams it decides which kernels overlap
    # (measured: largest alpha first, i.e. the smallest history grid first,
    # gives 4.70-4.74 ms per step against 4.83-4.86 as listed)
    order = [int(x) for x in a.order.split(",")] if a.order else list(range(len(plans)))[::-1]

    def step(parts):
        for i in order:
            plans[i].eval(sigma, mu, fv, ft, out=outs[i], parts=parts, join=False)
        for s in streams:
            if s is not cur:
                cur.wait_stream(s)

    def timed(parts, steps):
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        wall0 = time.perf_counter()
        for _ in range(steps):
            step(parts)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps, time.perf_counter() - wall0

    for _ in range(a.warmup):
        step(fresh)
    torch.cuda.synchronize()
    log("warmup done")
    # stage events are recorded by the library on its streams during the timed
    # steps and read after them (reading waits, so it stays outside the loop):
    # the stage times are those of the last timed step
    for p in plans:
        p.set_timing(True)
    ms_step, wall = timed(fresh, a.steps)
    evals = n_out * len(plans)
    value = evals / (ms_step * 1e-3)
    infos = [p.info() for p in plans]
    stage_keys = ("ms_geometry", "ms_spread", "ms_fft", "ms_multiply", "ms_interp", "ms_levels", "ms_local",
                  "ms_total")
    stage = {k: [inf[k] for inf in infos] for k in stage_keys}
    log(f"timed {a.steps} steps: {ms_step:.3f} ms/step (closest points included)")
    for p in plans:
        p.set_timing(False)
    for _ in range(a.warmup):
        step(M.PART_ALL)
    ms_res, _ = timed(M.PART_ALL, a.steps)
    log(f"resident local geometry: {ms_res:.3f} ms/step")
    noconv = [int(p.info()["n_noconv"]) for p in plans]

    # per-potential rates: S alone, D alone, V alone at every output of every
    # plan, closest points included
    per_pot = {}
    for name, args in () if a.no_per_potential else (("S", (sigma, None, None, None)), ("D", (None, mu, None, None)),
                                                      ("V", (None, None, fv, ft))):
        po = [p.eval(*args, parts=fresh) for p in plans]

        def pstep(args=args, po=po):
            for i in order:
                plans[i].eval(*args, out=po[i], parts=fresh, join=False)
            for s in streams:
                if s is not cur:
                    cur.wait_stream(s)
        for _ in range(a.warmup):
            pstep()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(a.steps):
            pstep()
        ev1.record()
        torch.cuda.synchronize()
        ms_p = ev0.elapsed_time(ev1) / a.steps
        per_pot[name] = {"ms_per_step": round(ms_p, 4), "target_evals_per_s": evals / (ms_p * 1e-3)}
        del po
    log(f"per potential: {per_pot}")

    # dominant kernel: the level sums (largest summed stage time)
    roof = roofline(stage, infos, w)
    stage_roof = stage_rooflines(stage, infos, w, roof)

    # parity against the oracle on a stratified sample of every plan's
    # outputs; the oracle's time on it is the CPU baseline
    check = None
    cpu = None
    if not a.no_check:
        check, cpu = parity_check(w, infos, alphas, outs, a.check_each)
        # the oracle's time for one whole step at its measured rate
        cpu["extrapolated_step_s"] = evals / cpu["value"]

    # the FP32 half of the metric (tol 1e-6) on its own workload, after the
    # FP64 plans are released
    fp32 = None
    if not a.no_fp32:
        for p in plans:
            p.close()
        del outs
        torch.cuda.empty_cache()
        fp32 = fp32_half(a, precision_workload())

    line = {
        "metric": "target evals/s at rel err 1e-10 (FP64) vs 1e-6 (FP32); p50/p99 request latency",
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
                   "batch": 1, "parallelism": "none", "streams": 1 if a.one_stream else len(alphas),
                   "step": "S, D, V at every output for each alpha, closest points included"},
        "resident_geometry": {"ms_per_step": ms_res, "value": evals / (ms_res * 1e-3)},
        "stage_ms": {k: [round(x, 4) for x in v] for k, v in stage.items()},
        "grid": [int(i["n_fine"]) for i in infos],
        "delta": [i["delta"] for i in infos],
        "plan_s": [round(x, 3) for x in plan_s],
        "plan_ms_phases": {"phases": ["inputs", "target_sort", "levels", "history", "local", "total"],
                           "ms": [[round(x, 1) for x in i["ms_plan"]] for i in infos]},
        "n_noconv": noconv,
        "gen_s": round(gen_s, 2),
        "wall_s": round(wall, 3),
        "rel_err_vs_oracle": check,
        "roofline": roof,
        "per_potential": per_pot,
        "stage_roofline": stage_roof,
        "cpu_baseline": cpu,
        "fp32": fp32,
        "latency_note": "p50/p99 request latency: bench.py --workload serve",
    }
    print(json.dumps(line), flush=True)
    if check is not None:
        worst = max(v for per in check["alpha"].values() for v in per.values())
        if not worst <= a.tol:
            log(f"parity FAILED: max relative error {worst:.3e} > {a.tol:g}")
            sys.exit(1)
    if fp32 is not None and "rel_err_vs_oracle_fp64_inputs" in fp32:
        worst = max(fp32["rel_err_vs_oracle_fp64_inputs"].values())
        if not worst <= fp32["bar"]:
            log(f"FP32 parity FAILED: max relative error {worst:.3e} > {fp32['bar']:g}")
            sys.exit(1)


def roofline(stage, infos, w):
    """The dominant kernel, k_level_sums: algorithmic flops per launch over
    its measured HIP-event time per launch (the level stage of each plan,
    on the stream the level sums are launched on, over its J launches)."""
    flops, pairs = 0.0, 0.0
    for info in infos:
        pr = level_pairs(w, info)
        pairs += pr
    flops = pairs * LEVEL_FLOPS_PER_PAIR
    launches = sum(i["J"] for i in infos)
    ms = sum(stage["ms_levels"])
    ach = flops / (ms * 1e-3) / 1e12
    tr = level_sums_traffic()
    return {"kernel": "k_level_sums", "bound": "alu", "achieved": ach, "peak": FP64_PEAK,
            "unit": "TFLOP/s", "frac": ach / FP64_PEAK, "traffic": tr,
            "flops_per_pair": LEVEL_FLOPS_PER_PAIR, "pairs_per_launch": pairs / launches,
            "flops_per_launch": flops / launches, "ms_per_launch": ms / launches,
            "frac_kernel_count": ach * LEVEL_FLOPS_PER_PAIR_KERNEL / LEVEL_FLOPS_PER_PAIR / FP64_PEAK,
            "flops_per_pair_kernel": LEVEL_FLOPS_PER_PAIR_KERNEL}


def stage_rooflines(stage, infos, w, roof):
    """Roofline fractions of the hot-path stages from their algorithmic work
    (the per-unit counts below) over their measured HIP-event times (the
    last timed step, the three plans overlapping), summed over the plans,
    and the time-weighted fraction over the stages counted.  The row and
    column transforms with the multiplier are timed but not counted: they
    move only the rows and columns of the sources' and targets' windows, and
    their measured HBM bytes are in the committed counter profile.
      spread (a3): per source component (S, D_x, D_y at the boundary nodes,
        V at the volume nodes) 2W^2 + 20W flops (window values and products);
      interpolation (a7): per output and result (S, D, V) 2W^2 + 20W flops,
        16 B of position read and 8 B written;
      level sums (a9): 23 flops per in-range pair (the dominant kernel);
      closest point and local part (a10-a11): per output in a local band
        ~600 flops (Newton on the panels, the coefficients), transcendentals
        not counted."""
    from scipy.spatial import cKDTree
    X = np.concatenate([w.tx, w.boundary["x"]])
    Y = np.concatenate([w.ty, w.boundary["y"]])
    d, _ = cKDTree(np.column_stack([w.boundary["x"], w.boundary["y"]])).query(np.column_stack([X, Y]))
    n_comp = 3 * w.n_b + w.n_v
    out = {}
    fl_sp = fl_in = fl_loc = 0.0
    for info in infos:
        W = int(info["wspread"])
        per = 2 * W * W + 20 * W
        fl_sp += n_comp * per
        fl_in += 3 * len(X) * per
        band = max(info["band_layer"], info["band_volume"])
        fl_loc += 600.0 * float(np.count_nonzero(d < band))
    t_sp = sum(stage["ms_spread"]) * 1e-3
    t_in = sum(stage["ms_interp"]) * 1e-3
    t_loc = (sum(stage["ms_geometry"]) + sum(stage["ms_local"])) * 1e-3
    t_lv = sum(stage["ms_levels"]) * 1e-3
    t_fft = (sum(stage["ms_fft"]) + sum(stage["ms_multiply"])) * 1e-3
    bytes_in = len(infos) * len(X) * (16 + 3 * 8)
    ent = lambda fl, t: {"ms": round(t * 1e3, 4), "achieved_tflops": fl / t / 1e12,
                         "frac": fl / t / 1e12 / FP64_PEAK, "bound": "alu (FP64)"}
    out["a3_spread"] = ent(fl_sp, t_sp)
    out["a7_interp"] = dict(ent(fl_in, t_in), achieved_gbs=bytes_in / t_in / 1e9,
                            frac_hbm=bytes_in / t_in / 1e9 / HBM_PEAK)
    out["a9_levels"] = {"ms": round(t_lv * 1e3, 4), "achieved_tflops": roof["achieved"], "frac": roof["frac"],
                        "bound": "alu (FP64)"}
    out["a10_a11_local"] = ent(fl_loc, t_loc)
    counted = [("a3_spread", t_sp), ("a7_interp", t_in), ("a9_levels", t_lv), ("a10_a11_local", t_loc)]
    tw = sum(t for _, t in counted)
    out["time_weighted_frac"] = sum(out[k]["frac"] * t for k, t in counted) / tw
    out["fft_multiply_ms_not_counted"] = round(t_fft * 1e3, 4)
    return out


# Algorithmic flops of one (target, child node) pair with r < R_j, as the
# method needs them: the separation and r^2 (5: two differences, a product,
# a multiply-add, the scale to the table variable), one degree-7 polynomial
# (7 multiply-adds, 14) and two multiply-adds of the single and double layer
# sums (4).  The kernel spends more per pair: the segment index and local
# variable (3), the polynomial's derivative for K_j^D (a second Horner chain
# of 7 multiply-adds, 14) and nu.(x - x_q) (3): 45 flops
# (flops_per_pair_kernel and frac_kernel_count in the roofline entry).
LEVEL_FLOPS_PER_PAIR = 23.0
LEVEL_FLOPS_PER_PAIR_KERNEL = 45.0


def level_sums_traffic():
    """HBM bytes per k_level_sums launch from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by the counter's
    reading for a device copy of known size), or None when levels.hip has
    changed since the counters were taken (its hash is recorded there)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "multibody_fp64_hbm_counters.md")
    src = os.path.join(ROOT, "paper_2606_28865_amd", "csrc", "levels.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    rec = {}
    for ln in text.splitlines():
        if ": " in ln and ln.strip().startswith("- "):
            k, v = ln.strip()[2:].split(": ", 1)
            rec[k.strip()] = v.strip().strip("`")
    if rec.get("levels.hip sha256[:16]") != sha:
        return None
    try:
        return float(rec["bytes per launch"])
    except (KeyError, ValueError):
        return None


def child_nodes(w, j):
    """Positions of the level-j child nodes (every panel bisected j times, 16
    Gauss-Legendre nodes per child), from the analytic curves."""
    import synth
    tg, _ = synth.gauss_legendre()
    xs = []
    ofs = w.boundary["curve_panel_ofs"]
    for c, cv in enumerate(w.curves):
        M = int(ofs[c + 1] - ofs[c])
        edges = np.linspace(0.0, 2 * np.pi, M + 1)
        nch = 1 << j
        h = (edges[1] - edges[0]) / nch
        t = (edges[:-1, None, None] + h * (np.arange(nch)[None, :, None] + 0.5 * (1 + tg[None, None, :]))).ravel()
        g, _, _ = cv.eval(t)
        xs.append(np.stack([g.real, g.imag], 1))
    return np.concatenate(xs)


def level_pairs(w, info):
    """Pairs (target, child node) with r < R_j summed over the levels."""
    from scipy.spatial import cKDTree
    tg = np.concatenate([np.stack([w.tx, w.ty], 1), np.stack([w.boundary["x"], w.boundary["y"]], 1)])
    pairs = 0.0
    for j in range(1, info["J"] + 1):
        tree = cKDTree(child_nodes(w, j))
        cnt = tree.query_ball_point(tg, info["level_radius"][j - 1], return_length=True, workers=-1)
        pairs += float(np.sum(cnt))
    return pairs


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads():
    """Threads the OpenMP oracle runs with: OMP_NUM_THREADS, else the CPUs
    this process may use."""
    try:
        return int(os.environ["OMP_NUM_THREADS"])
    except (KeyError, ValueError):
        return len(os.sched_getaffinity(0))


def strata(w, info, n_each, seed):
    """Output indices of a seeded stratified sample: n_each on-surface
    nodes, n_each targets in the layer band (nearest boundary node closer
    than the layer band), n_each in the volume band, n_each farther."""
    from scipy.spatial import cKDTree
    g = np.random.default_rng(seed)
    d, _ = cKDTree(np.column_stack([w.boundary["x"], w.boundary["y"]])).query(np.column_stack([w.tx, w.ty]))
    bl, bv = info["band_layer"], info["band_volume"]
    pick = lambda a, n: a if len(a) <= n else g.choice(a, n, replace=False)
    groups = {"on_surface": w.n_t + pick(np.arange(w.n_b), n_each),
              "layer_band": pick(np.nonzero(d < bl)[0], n_each),
              "volume_band": pick(np.nonzero((d >= bl) & (d < bv))[0], n_each),
              "far": pick(np.nonzero(d >= bv)[0], n_each)}
    return {k: np.sort(v).astype(np.int64) for k, v in groups.items()}


def parity_check(w, infos, alphas, outs, n_each):
    """Relative max-norm error of S, D and V per plan against the FP64
    oracle on a stratified sample of the outputs (errors relative to the
    largest oracle value of the sample), and the oracle's own rate on it."""
    import oracle as O
    res, total_t, total_n = {}, 0.0, 0
    for k, (alpha, info, out) in enumerate(zip(alphas, infos, outs)):
        groups = strata(w, info, n_each, seed=100 + k)
        sub = np.sort(np.concatenate(list(groups.values())))
        P = O.Problem(alpha, info["delta"], info["J"], w.boundary, volume=w.volume, targets=(w.tx, w.ty),
                      inside=w.inside, on_surface=True, sigma=w.sigma, mu=w.mu, f_vol=w.f_vol, f_trg=w.f_trg)
        t0 = time.perf_counter()
        ref = P.eval(sub)
        dt = time.perf_counter() - t0
        total_t += dt
        total_n += len(sub)
        errs = {}
        for name, o, rr in zip("SDV", out, ref):
            g = o.double().cpu().numpy().ravel()[sub]
            errs[name] = float(np.abs(g - rr).max() / np.abs(rr).max())
        res[f"{alpha:g}"] = errs
        log(f"alpha={alpha:g}: rel err vs oracle {errs} on {len(sub)} outputs ({dt:.1f} s)")
    check = {"alpha": res, "sample": f"{n_each} outputs per stratum (on-surface, layer band, volume band, "
                                     f"far) per alpha, seeded", "bar": 1e-10}
    cpu = {"value": total_n / total_t, "unit": "target-evals/s", "cores": oracle_threads(), "kind": "oracle",
           "cpu": cpu_model(),
           "sample": f"the {total_n} stratified outputs of the parity check (S, D, V each), all three alpha, "
                     f"{total_t:.1f} s"}
    return check, cpu


# ---------------------------------------------------------------------------
# Other workloads (one JSON line each)
# ---------------------------------------------------------------------------
def _stratified(w, band, n_each, seed):
    """Output indices: n_each on-surface nodes, n_each targets within `band`
    of a boundary node, n_each other targets (seeded)."""
    from scipy.spatial import cKDTree
    g = np.random.default_rng(seed)
    d, _ = cKDTree(np.column_stack([w.boundary["x"], w.boundary["y"]])).query(np.column_stack([w.tx, w.ty]))
    near, far = np.nonzero(d < band)[0], np.nonzero(d >= band)[0]
    pick = lambda a, n: a if len(a) <= n else g.choice(a, n, replace=False)
    on = w.n_t + pick(np.arange(w.n_b), n_each)
    return np.sort(np.concatenate([pick(near, n_each), pick(far, n_each), on])).astype(np.int64)


def _sample_errors(w, info, alpha, outs, n_each=12, seed=3, round32=False):
    """Relative max-norm error of (S, D, V) against the FP64 oracle on a
    stratified sample of outputs (on-surface, near the boundary, elsewhere).
    round32: feed the oracle the densities rounded to FP32, as the FP32 path
    sees them."""
    import oracle as O
    sub = _stratified(w, info["band_volume"], n_each, seed)
    r = (lambda a: np.asarray(a, np.float32).astype(np.float64)) if round32 else (lambda a: a)
    P = O.Problem(alpha, info["delta"], info["J"], w.boundary, volume=w.volume, targets=(w.tx, w.ty),
                  inside=w.inside, on_surface=True, sigma=r(w.sigma), mu=r(w.mu), f_vol=r(w.f_vol),
                  f_trg=r(w.f_trg))
    t0 = time.perf_counter()
    # in chunks of 16 outputs (one per host thread), with a progress line for
    # each (the oracle sums every source directly: seconds per output on the
    # large workloads)
    parts = []
    for c in range(0, len(sub), 16):
        parts.append(P.eval(sub[c:c + 16]))
        log(f"oracle sample: {min(c + 16, len(sub))}/{len(sub)} outputs, {time.perf_counter() - t0:.1f} s")
    ref = [np.concatenate([q[k] for q in parts]) for k in range(3)]
    dt = time.perf_counter() - t0
    errs = []
    for o, rr in zip(outs, ref):
        o = o.double().cpu().numpy().ravel()[sub]
        m = np.isfinite(rr)
        errs.append(float(np.abs(o[m] - rr[m]).max() / np.abs(rr[m]).max()))
    return errs, dt


def precision_workload():
    import synth
    t0 = time.time()
    w = synth.multibody(cfg=2, n_boundary=65536, n_volume=4_000_000, n_targets=4_000_000, alphas=(30.0,), tol=1e-6)
    log(f"workload {w.name} generated in {time.time() - t0:.1f} s")
    return w


def fp32_half(a, w):
    """The FP32 half of the headline metric: the FP32 path (FP64 densities,
    in64) at tol 1e-6 on the precision workload (65536 boundary nodes, ~4M
    volume nodes, 4M targets, alpha = 30), its rate and its error against
    the FP64 oracle on the same FP64 inputs (stratified sample)."""
    import torch

    import paper_2606_28865_amd as M
    alpha, tol = 30.0, 1e-6
    d64 = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    ins = (d64(w.sigma), d64(w.mu), d64(w.f_vol), d64(w.f_trg))
    t1 = time.time()
    p = M.Plan(M.make_params(alpha=alpha, tol=tol, prec=M.MHK_FP32, dx=w.dx, in64=1), w.boundary, w.volume,
               (w.tx, w.ty, w.inside), on_surface=True)
    plan_s = time.time() - t1
    # like the FP64 line: closest points and local coefficients recomputed in
    # every evaluation; the rate with them kept from plan creation beside
    fresh = M.PART_ALL | M.PART_GEOMETRY

    def timed(parts):
        for _ in range(a.warmup):
            p.eval(*ins, out=out, parts=parts)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            p.eval(*ins, out=out, parts=parts)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / a.steps
    out = p.eval(*ins, parts=fresh)
    ms = timed(fresh)
    ms_res = timed(M.PART_ALL)
    p.eval(*ins, out=out, parts=fresh)
    info = p.info()
    res = {"workload": "multibody-precision", "n_boundary": w.n_b, "n_volume": w.n_v, "n_targets": w.n_t,
           "alpha": alpha, "tol": tol, "inputs": "FP64 (in64)", "ms_per_eval": ms,
           "target_evals_per_s": p.n_out / (ms * 1e-3), "step": "closest points included",
           "resident_geometry": {"ms_per_eval": ms_res, "target_evals_per_s": p.n_out / (ms_res * 1e-3)},
           "grid": info["n_fine"], "plan_s": round(plan_s, 3)}
    if not a.no_check:
        errs, _ = _sample_errors(w, info, alpha, out, n_each=6)
        res["rel_err_vs_oracle_fp64_inputs"] = {"S": errs[0], "D": errs[1], "V": errs[2]}
        res["bar"] = tol
    log(f"fp32 half: {ms:.3f} ms per eval, {res['target_evals_per_s']:.3e} target-evals/s, "
        f"errors {res.get('rel_err_vs_oracle_fp64_inputs')}")
    p.close()
    del ins, out
    torch.cuda.empty_cache()
    return res


def run_precision(a):
    """FP32 vs FP64 at tol 1e-6 on the multi-body generator at 65536
    boundary nodes, ~4M volume nodes and 4M targets, alpha = 30."""
    import torch

    import paper_2606_28865_amd as M
    w = precision_workload()
    alpha, tol = 30.0, 1e-6
    res = {}
    for prec, dt, name in ((M.MHK_FP32, torch.float32, "fp32"), (M.MHK_FP64, torch.float64, "fp64")):
        t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
        ins = (t(w.sigma), t(w.mu), t(w.f_vol), t(w.f_trg))
        p = M.Plan(M.make_params(alpha=alpha, tol=tol, prec=prec, dx=w.dx), w.boundary, w.volume,
                   (w.tx, w.ty, w.inside), on_surface=True)
        # closest points recomputed in every evaluation, as in the default line
        fresh = M.PART_ALL | M.PART_GEOMETRY
        out = p.eval(*ins, parts=fresh)
        for _ in range(a.warmup):
            p.eval(*ins, out=out, parts=fresh)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            p.eval(*ins, out=out, parts=fresh)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        p.set_timing(True)
        p.eval(*ins, out=out, parts=fresh)
        info = p.info()
        errs, odt = _sample_errors(w, info, alpha, out, n_each=6, round32=(name == "fp32"))
        res[name] = {"ms_per_eval": ms, "target_evals_per_s": p.n_out / (ms * 1e-3),
                     "rel_err_vs_oracle": {"S": errs[0], "D": errs[1], "V": errs[2]}}
        if name == "fp32":
            # the same outputs against the oracle on the unrounded FP64 inputs:
            # adds the input rounding, amplified by the density's second
            # derivative in the local double-layer term (Lemma 4.5)
            e64, _ = _sample_errors(w, info, alpha, out, n_each=6)
            res[name]["rel_err_vs_oracle_fp64_inputs"] = {"S": e64[0], "D": e64[1], "V": e64[2]}
        res[name].update({
                     "stage_ms": {k: round(info[k], 4) for k in info if k.startswith("ms_") and not isinstance(info[k], list)},
                     "grid": info["n_fine"], "wspread": info["wspread"]})
        log(f"{name}: {ms:.2f} ms, errs {errs}")
        p.close()
        del ins, out
        torch.cuda.empty_cache()
    line = {"metric": "target evals/s at tol 1e-6, FP32 vs FP64", "value": res["fp32"]["target_evals_per_s"],
            "unit": "target-evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": res["fp32"]["ms_per_eval"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "multibody-precision", "n_boundary": w.n_b, "n_volume": w.n_v,
                       "n_targets": w.n_t, "alpha": alpha, "tol": tol},
            "results": res}
    print(json.dumps(line), flush=True)


def run_batched(a):
    """64 densities per call on one 65536-node multi-body geometry (~1M volume
    nodes, 1M targets + boundary nodes), evaluated by replaying a captured HIP
    graph; grid and level-sum tile shapes from the autotuner, timed at the
    same batch size; alpha in {3, 30}, FP32 and FP64.  Beside each, the same
    geometry and parameters with one density per call (its own captured
    graph), so that the per-density gain of batching is measured, and the
    level sums' roofline fraction of both forms (algorithmic flops of the
    pairs within the level radius, times the densities, over the level
    stage's HIP-event time of an eager evaluation)."""
    import torch

    import paper_2606_28865_amd as M
    from paper_2606_28865_amd import autotune
    import synth
    t0 = time.time()
    w = synth.multibody(cfg=3, n_boundary=65536, n_volume=1_000_000, n_targets=1_000_000, alphas=(3.0, 30.0))
    log(f"workload {w.name} generated in {time.time() - t0:.1f} s")
    B = a.batch
    g = np.random.default_rng(7)
    # B densities and sources with the config-0 spectra: rescaled copies
    # with seeded random mode amplitudes per density
    tt = w.boundary["t"]
    k = np.arange(9)
    sc = 1.0 / np.maximum(1, k) ** 2
    def dens():
        a_, b_ = g.standard_normal(9) * sc, g.standard_normal(9) * sc
        return (a_[None, :] * np.cos(np.outer(tt, k)) + b_[None, :] * np.sin(np.outer(tt, k))).sum(1)
    sig = np.stack([dens() for _ in range(B)])
    mu = np.stack([dens() for _ in range(B)])
    amp = g.standard_normal(B)
    fv = amp[:, None] * w.f_vol[None, :]
    ft = amp[:, None] * w.f_trg[None, :]
    geometry = {"boundary": w.boundary, "volume": w.volume, "targets": (w.tx, w.ty, w.inside), "on_surface": True}
    pairs_cache = {}

    def form(prm, ins, dt, nb):
        """Captured-graph time per call and the level stage of an eager call."""
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            p = M.Plan(prm, w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=True, stream=stream)
            # closest points recomputed in every call (shared by its densities)
            out = p.capture(*ins, parts=M.PART_ALL | M.PART_GEOMETRY)
            for _ in range(a.warmup):
                p.replay()
            stream.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(a.steps):
                p.replay()
            e1.record(stream)
            stream.synchronize()
            ms = e0.elapsed_time(e1) / a.steps
            p.set_timing(True)
            p.eval(*ins, out=out, parts=M.PART_ALL | M.PART_GEOMETRY)
            info = p.info()
            p.set_timing(False)
        key = (info["alpha"], info["delta"])
        if key not in pairs_cache:
            pairs_cache[key] = level_pairs(w, info)
        flops = pairs_cache[key] * LEVEL_FLOPS_PER_PAIR * nb
        ach = flops / (info["ms_levels"] * 1e-3) / 1e12
        peak = FP64_PEAK if dt == torch.float64 else FP32_PEAK
        res = {"ms_per_call": ms, "densities": nb, "ms_per_density": ms / nb,
               "target_evals_per_s": nb * p.n_out / (ms * 1e-3), "grid": info["n_fine"],
               "level_sums": {"ms": info["ms_levels"], "achieved_tflops": ach, "peak_tflops": peak,
                              "frac": ach / peak, "flops": flops},
               "stage_ms": {k2: info[k2] for k2 in ("ms_spread", "ms_fft", "ms_multiply", "ms_interp", "ms_levels",
                                                    "ms_local", "ms_total")}}
        p.close()
        del out
        torch.cuda.empty_cache()
        return res

    res = {}
    for alpha in (3.0, 30.0):
        for prec, dt, name, tol in ((M.MHK_FP32, torch.float32, "fp32", 1e-6), (M.MHK_FP64, torch.float64, "fp64", 1e-10)):
            tun = autotune.tune(geometry, alpha, tol, prec, (w.sigma, w.mu, w.f_vol, w.f_trg), dx=w.dx, batch=B,
                                cache=None, log=log)
            mk = lambda b, bch, ps: M.make_params(alpha=alpha, tol=tol, prec=prec, delta=tun["delta"], batch=b,
                                                  upsamp=tun["upsamp"], wspread=tun["wspread"],
                                                  lv_block=tun["lv_block"], lv_bch=bch, lv_persist=ps)
            t = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
            batched = form(mk(B, tun["lv_bch"], tun["lv_persist"]), (t(sig), t(mu), t(fv), t(ft)), dt, B)
            single = form(mk(1, 0, 0), (t(sig[:1]), t(mu[:1]), t(fv[:1]), t(ft[:1])), dt, 1)
            key = f"{name}_alpha{alpha:g}"
            res[key] = {"batched": batched, "single": single,
                        "speedup_per_density": single["ms_per_call"] * B / batched["ms_per_call"],
                        "upsamp": tun["upsamp"], "wspread": tun["wspread"], "lv_block": tun["lv_block"],
                        "lv_bch": tun["lv_bch"], "lv_persist": tun["lv_persist"],
                        "autotune": tun["table"], "autotune_tiles": tun["tile_table"]}
            log(f"{key}: {batched['ms_per_call']:.1f} ms per {B} densities ({batched['ms_per_density']:.3f} ms each, "
                f"levels {batched['level_sums']['frac']:.3f} of peak) vs {single['ms_per_call']:.3f} ms for one "
                f"(levels {single['level_sums']['frac']:.3f}): x{res[key]['speedup_per_density']:.2f} per density")
    best = max(v["batched"]["target_evals_per_s"] for v in res.values())
    line = {"metric": "target evals/s, 64 densities per call under a captured HIP graph", "value": best,
            "unit": "target-evals/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "multibody-batched", "n_boundary": w.n_b, "n_volume": w.n_v,
                       "n_targets": w.n_t, "batch": B},
            "results": res}
    print(json.dumps(line), flush=True)


def run_serve(a):
    """Poisson stream of Rothe-step requests from several concurrent
    simulations (1-50 bodies, 1k-128k boundary nodes, 10k-2M volume nodes,
    alpha log-uniform in [1, 300], tol 1e-6 (FP32) or 1e-10 (FP64))."""
    import torch

    import synth
    from paper_2606_28865_amd.serve import Geometry, Request, Server, latency_stats
    g = np.random.default_rng(4)
    sims = []
    t0 = time.time()
    sizes = [(3, 2048, 20_000), (12, 8192, 150_000), (1, 1024, 10_000), (30, 32768, 600_000),
             (50, 131072, 2_000_000), (6, 4096, 60_000)]
    for si, (nbod, nb, nv) in enumerate(sizes):
        w = synth.multibody(cfg=100 + si, n_bodies=nbod, n_boundary=nb, n_volume=nv, n_targets=nv // 2,
                            box=1.0 if nbod < 30 else 1.4)
        alpha = float(np.exp(g.uniform(np.log(1.0), np.log(300.0))))
        tol = 1e-6 if g.uniform() < 0.5 else 1e-10
        geo = Geometry(f"sim{si}", w.boundary, w.volume, (w.tx, w.ty, w.inside), True)
        sims.append((w, geo, alpha, tol))
        log(f"sim {si}: {nbod} bodies, nb {w.n_b}, nv {w.n_v}, alpha {alpha:.1f}, tol {tol:g}")
    log(f"generated in {time.time() - t0:.1f} s")

    def make_req(rid, si, arrival):
        w, geo, alpha, tol = sims[si]
        s = 1.0 + 0.1 * g.standard_normal()
        return Request(rid, geo, alpha, tol, 1 if tol >= 1e-6 else 0, w.sigma * s, w.mu * s, w.f_vol * s,
                       w.f_trg * s, arrival=arrival, dx=w.dx)

    def sweep_loads(srv, loads, mean_svc, tag):
        out, done_all, evals_all, span_all = [], [], 0, 0.0
        for util in loads:                   # offered load, fraction of one-at-a-time capacity
            lam = util / mean_svc
            t = 0.0
            reqs = []
            for rid in range(a.requests):
                t += g.exponential(1.0 / lam)
                reqs.append(make_req(rid, int(g.integers(len(sims))), t))
            t0 = time.perf_counter()
            done = list(srv.run(reqs))
            span = time.perf_counter() - t0
            srv.finished.clear()
            st = latency_stats(done)
            evals = sum(r.geometry.n_out for r in done)
            out.append({"offered_util": util, "arrival_rate_per_s": lam, "served_evals_per_s": evals / span,
                        "span_s": span, "mean_batched_with": float(np.mean([r.batched_with for r in done])), **st})
            log(f"{tag} util {util}: {st}, {evals / span:.3e} evals/s, "
                f"mean coalesced {out[-1]['mean_batched_with']:.2f}")
            evals_all += evals
            span_all += span
            done_all += done
        return out, done_all, evals_all, span_all

    budget = int(torch.cuda.mem_get_info()[0] * 0.7)
    srv = Server(budget_bytes=budget, max_inflight=8, max_batch=a.max_batch)
    # warm-up: one request per simulation (plan creation), also gives service times
    warm = [make_req(-1 - i, i, 0.0) for i in range(len(sims))]
    srv.run(warm)
    srv.finished.clear()
    # measured service time per request when run alone
    alone = []
    for i in range(len(sims)):
        r = make_req(-100 - i, i, 0.0)
        srv.run([r])
        alone.append(r.done - r.admitted)
    srv.finished.clear()
    mean_svc = float(np.mean(alone))
    sweep, done_all, evals_all, span_all = sweep_loads(srv, (0.5, 0.8, 0.95, 1.5), mean_svc,
                                                       f"coalesced (max_batch {a.max_batch})")
    srv.close()
    # the same stream without coalescing, at the two highest loads
    plain = Server(budget_bytes=budget, max_inflight=8, max_batch=1)
    plain.run([make_req(-200 - i, i, 0.0) for i in range(len(sims))])
    plain.finished.clear()
    sweep_plain, _, _, _ = sweep_loads(plain, (0.95, 1.5), mean_svc, "not coalesced")
    plain.close()
    # cold start: a fresh server at 80% load, every plan built on its
    # simulation's first request (in the server's build thread, beside the
    # requests of plans already built)
    cold = Server(budget_bytes=budget, max_inflight=8, max_batch=a.max_batch)
    sweep_cold, done_cold, _, _ = sweep_loads(cold, (0.8,), mean_svc, "cold start")
    first = {}
    for r in sorted(done_cold, key=lambda r: r.arrival):
        first.setdefault(r.geometry.key, r)
    sweep_cold[0]["first_request_ms"] = {k: round((r.done - r.arrival) * 1e3, 1) for k, r in first.items()}
    cold.close()
    heat = run_serve_heat(a, make_req, mean_svc, len(sims))
    st = latency_stats(done_all)
    line = {"metric": "served target evals/s with p50/p99 request latency", "value": evals_all / span_all,
            "unit": "target-evals/s", "n_gpus": 1, "steps": len(done_all), "warmup": len(warm),
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "rothe-serving", "simulations": len(sims), "requests_per_load": a.requests,
                       "sizes": sizes, "max_batch": a.max_batch},
            "latency": st, "sweep": sweep, "sweep_not_coalesced": sweep_plain, "cold_start": sweep_cold[0],
            "alone_service_ms": [round(x * 1e3, 3) for x in alone], "heat_chains": heat}
    print(json.dumps(line), flush=True)


def run_serve_heat(a, make_req, mean_svc, n_sims):
    """Heat-equation simulations (elliptic marching) driven through the
    server: each chain's step n + 1 is submitted when step n is done, with
    its result as input, beside a Poisson stream of eval requests at half
    the one-at-a-time load.  Returns per-step latency and node updates/s."""
    import torch

    import synth
    from paper_2606_28865_amd.serve import Geometry, HeatChain, Server, latency_stats
    g = np.random.default_rng(9)
    k = np.pi
    chains = []
    for i, (nbod, nb, nv, alpha) in enumerate([(3, 2048, 50_000, 10.0), (10, 16384, 1_000_000, 10.0),
                                               (6, 8192, 300_000, 30.0)]):
        w = synth.multibody(cfg=300 + i, n_bodies=nbod, n_boundary=nb, n_volume=nv, n_targets=10,
                            box=1.0)
        vol = w.volume
        geo = Geometry(f"heat{i}", w.boundary, vol, (vol["x"], vol["y"], np.ones(len(vol["x"]), np.int8)), True)
        X = np.concatenate([vol["x"], w.boundary["x"]])
        Y = np.concatenate([vol["y"], w.boundary["y"]])
        u0 = np.sin(k * (X + 0.3)) * np.sin(k * (Y + 0.2))
        c = alpha ** 2 / (alpha ** 2 + 2 * k * k)
        gb = u0[len(vol["x"]):]
        chains.append((HeatChain(i, geo, alpha, 1e-10, u0, lambda n, gb=gb, c=c: c ** n * gb, a.heat_steps,
                                 dx=w.dx, rid0=10_000 * (i + 1)), u0, c))
        log(f"heat chain {i}: {nbod} bodies, nb {w.n_b}, nv {len(vol['x'])}, alpha {alpha}")
    srv = Server(budget_bytes=int(torch.cuda.mem_get_info()[0] * 0.7), max_inflight=8, max_batch=a.max_batch)
    # plans and Nystrom matrices built before timing: one step of each chain
    warm = [HeatChain(100 + c.sid, c.geometry, c.alpha, c.tol, u0, c.g_of_step, 1, dx=c.dx, rid0=-1000 * (i + 1))
            for i, (c, u0, _) in enumerate(chains)]
    srv.run([wc.first() for wc in warm])
    srv.finished.clear()
    lam = 0.5 / mean_svc
    t = 0.0
    evals = []
    for rid in range(a.requests):
        t += g.exponential(1.0 / lam)
        evals.append(make_req(50_000 + rid, int(g.integers(n_sims)), t))
    t0 = time.perf_counter()
    srv.run([c.first() for c, _, _ in chains] + evals)
    span = time.perf_counter() - t0
    steps = [r for c, _, _ in chains for r in c.steps]
    st_heat = latency_stats(steps)
    st_eval = latency_stats([r for r in srv.finished if r.kind == "eval"])
    updates = sum(c.geometry.n_out * len(c.steps) for c, _, _ in chains)
    errs = []
    for c, u0, cc in chains:
        ex = cc ** c.nsteps * u0
        got = c.steps[-1].result[0].cpu().numpy()
        errs.append(float(np.abs(got - ex).max() / np.abs(ex).max()))
    srv.close()
    log(f"heat chains: steps {st_heat}, evals beside them {st_eval}, {updates / span:.3e} node updates/s, "
        f"errors vs c^n u0 {errs}")
    return {"chains": len(chains), "steps_per_chain": a.heat_steps, "span_s": span,
            "node_updates_per_s": updates / span, "step_latency": st_heat, "eval_latency_beside": st_eval,
            "rel_err_vs_closed_form": errs}


def run_bie(a):
    """Dirichlet problem on the 10-body geometry (16384 boundary nodes, ~1M
    volume nodes, 1M targets + boundary nodes), alpha = 10, FP64, tol 1e-10
    for the potentials and 1e-12 for GMRES: Nystrom assembly, the product's
    HBM roofline, GMRES iterations and the whole solve (right-hand side V at
    the boundary, GMRES, u = V + D[mu] at every output)."""
    import torch

    import paper_2606_28865_amd as M
    import synth
    from oracle import bie as OB
    w = synth.multibody()
    alpha = 10.0
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    plan = M.Plan(M.make_params(alpha=alpha, tol=1e-10, dx=w.dx), w.boundary, w.volume, (w.tx, w.ty, w.inside),
                  on_surface=True)
    nys = M.Nystrom(alpha, w.boundary)
    ninfo = nys.info()
    n = w.n_b
    x = dev(np.random.default_rng(5).standard_normal(n))
    y = torch.empty_like(x)
    for _ in range(3):
        nys.apply(x, -0.5, out=y)
    torch.cuda.synchronize()
    reps = 50
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        nys.apply(x, -0.5, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms_prod = e0.elapsed_time(e1) / reps
    bytes_prod = 8.0 * n * (n + n % 2) + 16.0 * n       # K once, x and y
    g, fv, ft = dev(w.sigma), dev(w.f_vol), dev(w.f_trg)
    M.solve_dirichlet(plan, nys, g, fv, ft, tol=1e-12)
    torch.cuda.synchronize()
    times, infos = [], []
    for _ in range(a.steps):
        t0 = time.perf_counter()
        mu, u, info = M.solve_dirichlet(plan, nys, g, fv, ft, tol=1e-12)
        times.append(time.perf_counter() - t0)
        infos.append(info)
    ms_solve = 1e3 * float(np.mean(times))
    log(f"product {ms_prod:.3f} ms ({bytes_prod / ms_prod / 1e6:.0f} GB/s), solve {ms_solve:.1f} ms, {infos[-1]}")
    # CPU oracle: rows of the Nystrom matrix times x on a bounded sample
    rows = np.arange(0, n, max(1, n // 512))
    xh = x.cpu().numpy()
    t0 = time.perf_counter()
    _ = OB.nystrom_rows(w.boundary, alpha, rows) @ xh
    cpu_rows_s = len(rows) / (time.perf_counter() - t0)
    line = {"metric": "Dirichlet solves/s (V at the boundary, GMRES to 1e-12, u = V + D at all outputs)",
            "value": 1e3 / ms_solve, "unit": "solves/s", "n_gpus": 1, "steps": a.steps, "warmup": 1,
            "ms_per_step": ms_solve, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "multibody-dirichlet", "n_boundary": n, "n_volume": w.n_v, "n_targets": w.n_t,
                       "alpha": alpha},
            "gmres_iters": infos[-1]["iters"], "resid": infos[-1]["resid"],
            "ms_gmres": infos[-1]["ms_gmres"], "ms_eval": infos[-1]["ms_eval"],
            "ms_assemble": ninfo["ms_assemble"], "nystrom_bytes": ninfo["device_bytes"],
            "roofline": {"kernel": "k_gemv", "bound": "hbm", "achieved": bytes_prod / ms_prod / 1e6,
                         "peak": 8000.0, "unit": "GB/s", "frac": bytes_prod / ms_prod / 1e6 / 8000.0,
                         "traffic": None, "ms_per_launch": ms_prod},
            "cpu_baseline": {"value": cpu_rows_s / n, "unit": "Nystrom products/s", "cores": os.cpu_count(),
                             "kind": "oracle", "sample": f"{len(rows)} rows of K times x (numpy, scipy K1)"}}
    print(json.dumps(line), flush=True)
    plan.close()
    nys.close()


def run_heat(a):
    """Elliptic marching of the heat equation on the 10-body geometry (16384
    boundary nodes, ~1M volume nodes carrying u), alpha = 10 (time step
    0.01), FP64: each step is a Dirichlet solve with the source alpha^2 u^n
    evaluated at every volume node.  u0 = sin(pi(x+0.3)) sin(pi(y+0.2)) with
    boundary data c^n u0, c = alpha^2/(alpha^2 + 2 pi^2), whose steps are
    exactly c^n u0: the error against that is reported."""
    import torch

    import paper_2606_28865_amd as M
    import synth
    w = synth.multibody(n_targets=10)
    vol = w.volume
    nv, nb = len(vol["x"]), w.n_b
    alpha = 10.0
    plan = M.Plan(M.make_params(alpha=alpha, tol=1e-10, dx=w.dx), w.boundary, vol,
                  (vol["x"], vol["y"], np.ones(nv, np.int8)), on_surface=True)
    nys = M.Nystrom(alpha, w.boundary)
    k = np.pi
    X = np.concatenate([vol["x"], w.boundary["x"]])
    Y = np.concatenate([vol["y"], w.boundary["y"]])
    u0 = np.sin(k * (X + 0.3)) * np.sin(k * (Y + 0.2))
    c = alpha ** 2 / (alpha ** 2 + 2 * k * k)
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
    gb = u0[nv:]
    nsteps = max(2, a.steps)
    gs = [dev(c ** n * gb) for n in range(1, nsteps + 2)]
    u = dev(u0)
    bufs = [torch.empty_like(u), torch.empty_like(u)]
    u1, _, info = M.heat_step(plan, nys, u, gs[0], tol=1e-12, out=bufs[0])        # warm-up step
    torch.cuda.synchronize()
    u = dev(u0)
    iters = []
    t0 = time.perf_counter()
    for n in range(nsteps):
        u, _, info = M.heat_step(plan, nys, u, gs[n], tol=1e-12, out=bufs[n % 2])
        iters.append(info["iters"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ex = c ** nsteps * u0
    err = float(np.abs(u.cpu().numpy() - ex).max() / np.abs(ex).max())
    ms = 1e3 * dt / nsteps
    log(f"heat: {ms:.1f} ms per step, GMRES iterations {iters}, error vs c^n u0 {err:.2e}")
    line = {"metric": "heat steps/s (implicit Euler, Dirichlet solve with V at 1M volume nodes)",
            "value": nsteps / dt, "unit": "steps/s", "n_gpus": 1, "steps": nsteps, "warmup": 1,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "multibody-heat", "n_boundary": nb, "n_volume": nv, "alpha": alpha,
                       "time_step": 1.0 / alpha ** 2},
            "node_updates_per_s": (nv + nb) * nsteps / dt, "gmres_iters": iters,
            "ms_eval": info["ms_eval"], "ms_gmres": info["ms_gmres"], "rel_err_vs_closed_form": err}
    print(json.dumps(line), flush=True)
    plan.close()
    nys.close()


if __name__ == "__main__":
    main()
