"""Parity of the HIP path with the CPU FP64 oracle (same split sums, history
and levels summed directly in the oracle).

Tolerance: the FP64 path must match the oracle to a relative max-norm error
of 1e-10 per potential (max |gpu - oracle| / max |oracle|), the accuracy the
plan is built for (tol = 1e-10); the NaN pattern (V at exterior targets in
the volume band, which has no local formula) must match exactly.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from helpers import oracle_eval, rel_err, small_multibody, stratified_subset

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _M():
    import paper_2606_28865_amd as M
    return M


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _run(plan, w, sigma=None, mu=None, f_vol=None, f_trg=None, parts=7, batch=1):
    s = w.sigma if sigma is None else sigma
    m = w.mu if mu is None else mu
    fv = w.f_vol if f_vol is None else f_vol
    ft = w.f_trg if f_trg is None else f_trg
    out = plan.eval(_dev(s), _dev(m), _dev(fv), _dev(ft), parts=parts)
    torch.cuda.synchronize()
    return [o.cpu().numpy().reshape(batch, -1) for o in out]


@pytest.fixture(scope="module")
def cfg0():
    return synth.config0()


def _plan(w, alpha, tol=TOL, J=3, batch=1, on_surface=True, delta=0.0, **kw):
    M = _M()
    prm = M.make_params(alpha=alpha, tol=tol, dx=w.dx, J=J, batch=batch, delta=delta, **kw)
    return M.Plan(prm, w.boundary, w.volume, (w.tx, w.ty, w.inside), on_surface=on_surface)


def test_config0_full(cfg0):
    """Config 0 (starfish, 512 boundary nodes, cut-cell volume, 64x64 grid +
    boundary nodes), alpha = 10: S, D, V at every target."""
    w = cfg0
    print("case config0 alpha=10 all parts", flush=True)
    plan = _plan(w, 10.0)
    info = plan.info()
    S, D, V = _run(plan, w)
    So, Do, Vo = oracle_eval(w, 10.0, info["delta"], 3)
    es, ed, ev = rel_err(S, So), rel_err(D, Do), rel_err(V, Vo)
    print(f"config0 rel err S {es:.2e} D {ed:.2e} V {ev:.2e}", flush=True)
    assert es < TOL and ed < TOL and ev < TOL


@pytest.mark.parametrize("parts", [O.PART_HISTORY, O.PART_LEVELS, O.PART_LOCAL])
def test_config0_parts(cfg0, parts):
    """Each part of the split alone (history, dyadic levels, local)."""
    w = cfg0
    print(f"case config0 parts={parts}", flush=True)
    plan = _plan(w, 10.0)
    info = plan.info()
    S, D, V = _run(plan, w, parts=parts)
    So, Do, Vo = oracle_eval(w, 10.0, info["delta"], 3, parts=parts)
    scale = [np.nanmax(np.abs(x)) for x in oracle_eval(w, 10.0, info["delta"], 3)]
    for g, o, sc, name in ((S, So, scale[0], "S"), (D, Do, scale[1], "D"), (V, Vo, scale[2], "V")):
        g = g.ravel()
        m = np.isfinite(o)
        assert np.array_equal(m, np.isfinite(g)), name
        err = np.abs(g[m] - o[m]).max() / sc
        print(f"parts {parts} {name}: err/max|total| {err:.2e}", flush=True)
        assert err < TOL, (name, err)


@pytest.mark.parametrize("alpha", [1.0, 3.0, 30.0, 300.0])
def test_config0_alphas(cfg0, alpha):
    """Other alpha: small (truncated history kernel, tabulated spectrum),
    large (at 300 the history is below 1e-12 of its peak, Section 5.2)."""
    w = cfg0
    print(f"case config0 alpha={alpha}", flush=True)
    plan = _plan(w, alpha)
    info = plan.info()
    S, D, V = _run(plan, w)
    So, Do, Vo = oracle_eval(w, alpha, info["delta"], 3)
    errs = [rel_err(S, So), rel_err(D, Do), rel_err(V, Vo)]
    print(f"alpha {alpha} kmax {info['kmax']:.1f} n {info['n_fine']} trunc {info['history_truncated']} "
          f"errs {errs}", flush=True)
    assert max(errs) < TOL


@pytest.mark.parametrize("delta,lo,hi", [(1e-5, 4096, 8192), (2e-6, 8192, 1 << 30)])
def test_long_grid_transforms(cfg0, delta, lo, hi):
    """Long history grids: 4096 < n <= 8192 takes the LDS transforms with
    their second register sizing, n > 8192 (longer than a column the column
    kernel holds in LDS) rocFFT's 2D transforms with the separate multiplier
    kernel.  Config 0 at alpha = 10 with a small delta (k_max ~ 1700 or
    ~ 4000), the history part alone against the oracle's (relative
    max-norm)."""
    w = cfg0
    print(f"case config0 alpha=10 delta={delta} (long grid)", flush=True)
    plan = _plan(w, 10.0, delta=delta)
    info = plan.info()
    print(f"n {info['n_fine']}", flush=True)
    assert lo < info["n_fine"] <= hi
    S, D, V = _run(plan, w, parts=O.PART_HISTORY)
    So, Do, Vo = oracle_eval(w, 10.0, info["delta"], 3, parts=O.PART_HISTORY)
    for g, o, name in ((S, So, "S"), (D, Do, "D"), (V, Vo, "V")):
        err = rel_err(g.ravel(), o)
        print(f"long grid {name}: err {err:.2e}", flush=True)
        assert err < TOL, (name, err)
    plan.close()


def test_batch_matches_single(cfg0):
    """Three densities in one call equal three single calls (and the oracle)."""
    w = cfg0
    g = np.random.default_rng(3)
    B = 3
    sig = np.stack([w.sigma * (1 + 0.1 * k) + 0.05 * g.standard_normal(w.n_b) for k in range(B)])
    mu = np.stack([w.mu * (1 - 0.2 * k) for k in range(B)])
    fv = np.stack([w.f_vol * (k + 1) for k in range(B)])
    ft = np.stack([w.f_trg * (k + 1) for k in range(B)])
    print("case batch=3", flush=True)
    plan = _plan(w, 10.0, batch=B)
    S, D, V = _run(plan, w, sig, mu, fv, ft, batch=B)
    single = _plan(w, 10.0)
    for k in range(B):
        s1, d1, v1 = _run(single, w, sig[k], mu[k], fv[k], ft[k])
        assert rel_err(S[k], s1[0]) < 1e-14 and rel_err(D[k], d1[0]) < 1e-14 and rel_err(V[k], v1[0]) < 1e-14
    k = 2
    So, Do, Vo = oracle_eval(w, 10.0, plan.info()["delta"], 3, sigma=sig[k], mu=mu[k], f_vol=fv[k], f_trg=ft[k])
    assert rel_err(S[k], So) < TOL and rel_err(D[k], Do) < TOL and rel_err(V[k], Vo) < TOL


@pytest.mark.parametrize("lv_block", [256, 512])
def test_level_tile_shapes(cfg0, lv_block):
    """Every tile shape of the level sums (targets per workgroup, densities
    per pass, persistent launch or not) gives the same S and D, up to the order of the sums: five
    densities through each shape against one single-density plan, the last
    density against the oracle."""
    w = cfg0
    B = 5
    g = np.random.default_rng(11)
    sig = np.stack([w.sigma * (1 + 0.1 * k) + 0.05 * g.standard_normal(w.n_b) for k in range(B)])
    mu = np.stack([w.mu * (1 - 0.2 * k) for k in range(B)])
    single = _plan(w, 10.0)
    ref = [_run(single, w, sig[k], mu[k], None, None, parts=O.PART_LEVELS)[:2] for k in range(B)]
    for bch, pers in [(b, p) for p in (0, 1) for b in (1, 2, 4, 8)]:
        print(f"case level tiles lv_block={lv_block} lv_bch={bch} lv_persist={pers}", flush=True)
        plan = _plan(w, 10.0, batch=B, lv_block=lv_block, lv_bch=bch, lv_persist=pers)
        S, D, _ = _run(plan, w, sig, mu, np.zeros((B, w.n_v)), np.zeros((B, w.n_t + w.n_b)), parts=O.PART_LEVELS,
                       batch=B)
        for k in range(B):
            assert rel_err(S[k], ref[k][0][0]) < 1e-13 and rel_err(D[k], ref[k][1][0]) < 1e-13, (bch, pers, k)
        plan.close()
    plan = _plan(w, 10.0, batch=B, lv_block=lv_block, lv_bch=4)
    S, D, V = _run(plan, w, sig, mu, np.stack([w.f_vol] * B), np.stack([w.f_trg] * B), batch=B)
    k = B - 1
    So, Do, Vo = oracle_eval(w, 10.0, plan.info()["delta"], 3, sigma=sig[k], mu=mu[k])
    assert rel_err(S[k], So) < TOL and rel_err(D[k], Do) < TOL and rel_err(V[k], Vo) < TOL


def test_run_twice_reproducible(cfg0):
    w = cfg0
    print("case run twice", flush=True)
    plan = _plan(w, 10.0)
    a = _run(plan, w)
    b = _run(plan, w)
    for x, y in zip(a, b):
        assert rel_err(x, y) < 1e-15
    # levels and local part only: fixed summation order, bitwise equal
    a = _run(plan, w, parts=O.PART_LEVELS | O.PART_LOCAL)
    b = _run(plan, w, parts=O.PART_LEVELS | O.PART_LOCAL)
    for x, y in zip(a, b):
        assert np.array_equal(np.nan_to_num(x, nan=1e300), np.nan_to_num(y, nan=1e300))


def test_edge_cases(cfg0):
    """Boundary-only targets, J = 0 (no levels), no volume."""
    w = cfg0
    M = _M()
    print("case edge: on-surface targets only, J=0", flush=True)
    prm = M.make_params(alpha=10.0, tol=TOL, dx=w.dx, J=0)
    plan = M.Plan(prm, w.boundary, w.volume, (np.zeros(0), np.zeros(0), np.zeros(0, np.int8)), on_surface=True)
    ft = w.f_trg[w.n_t:]
    out = plan.eval(_dev(w.sigma), _dev(w.mu), _dev(w.f_vol), _dev(ft))
    torch.cuda.synchronize()
    P = O.Problem(10.0, plan.info()["delta"], 0, w.boundary, volume=w.volume, targets=(np.zeros(0), np.zeros(0)),
                  inside=np.zeros(0), on_surface=True, sigma=w.sigma, mu=w.mu, f_vol=w.f_vol, f_trg=ft)
    ref = P.eval()
    for g, o in zip(out, ref):
        assert rel_err(g.cpu().numpy(), o) < TOL
    print("case edge: no volume, S only", flush=True)
    prm = M.make_params(alpha=10.0, tol=TOL, dx=w.dx)
    plan = M.Plan(prm, w.boundary, None, (w.tx, w.ty, w.inside), on_surface=False)
    S, D, V = plan.eval(_dev(w.sigma))
    torch.cuda.synchronize()
    assert D is None and V is None
    So, _, _ = oracle_eval(w, 10.0, plan.info()["delta"], 3, on_surface=False, f_vol=np.zeros(w.n_v))
    assert rel_err(S.cpu().numpy(), So) < TOL


def test_single_target(cfg0):
    """One off-surface output (n_out = 1: a partial wavefront, workgroup and
    tile in every kernel): the interior target nearest the boundary, so that
    the level sums, the closest point and the layer and volume local terms
    all run for it."""
    from scipy.spatial import cKDTree
    w = cfg0
    M = _M()
    d, _ = cKDTree(np.column_stack([w.boundary["x"], w.boundary["y"]])).query(np.column_stack([w.tx, w.ty]))
    d = np.where(w.inside != 0, d, np.inf)
    k = int(np.argmin(d))
    tx, ty, ins, ft = w.tx[k:k + 1], w.ty[k:k + 1], w.inside[k:k + 1], w.f_trg[k:k + 1]
    print(f"case single target: index {k}, distance {d[k]:.2e}", flush=True)
    plan = M.Plan(M.make_params(alpha=10.0, tol=TOL, dx=w.dx), w.boundary, w.volume, (tx, ty, ins),
                  on_surface=False)
    assert plan.n_out == 1
    out = plan.eval(_dev(w.sigma), _dev(w.mu), _dev(w.f_vol), _dev(ft))
    torch.cuda.synchronize()
    P = O.Problem(10.0, plan.info()["delta"], 3, w.boundary, volume=w.volume, targets=(tx, ty), inside=ins,
                  on_surface=False, sigma=w.sigma, mu=w.mu, f_vol=w.f_vol, f_trg=ft)
    for g, o in zip(out, P.eval()):
        assert rel_err(g.cpu().numpy(), o) < TOL


@pytest.mark.parametrize("alpha,trunc", [(1.0, 1), (30.0, 0)])
def test_multibody_sampled(alpha, trunc):
    """Small multi-body workload (3 bodies, 2048 boundary nodes, ~40k volume
    nodes, 6000 targets) with the fine split delta = 2e-5 of the bench
    workload, oracle on a stratified target sample.  At alpha = 1 the history
    uses the smoothly truncated kernel, at alpha = 30 the periodic one."""
    w = small_multibody()
    print(f"case multibody alpha={alpha} nb={w.n_b} nv={w.n_v} nt={w.n_t}", flush=True)
    plan = _plan(w, alpha, delta=2e-5)
    info = plan.info()
    assert info["history_truncated"] == trunc
    S, D, V = _run(plan, w)
    sub = stratified_subset(w, info["band_volume"])
    So, Do, Vo = oracle_eval(w, alpha, info["delta"], 3, subset=sub)
    errs = [rel_err(S[0][sub], So), rel_err(D[0][sub], Do), rel_err(V[0][sub], Vo)]
    print(f"multibody errs {errs} n {info['n_fine']}", flush=True)
    assert max(errs) < TOL


def test_exterior_volume_targets():
    """V at exterior targets near the boundary (complement-domain form of the
    local part, f taken at the closest boundary point from f at the boundary
    nodes), with two densities of different sources per call: targets along
    the outward normals of config 0's starfish at distances 1e-4 .. 0.3."""
    import paper_2606_28865_amd as M
    w = synth.config0()
    print("case exterior V targets config0 batch 2", flush=True)
    t0 = np.linspace(0.05, 2 * np.pi, 40, endpoint=False)
    g, g1, _ = w.curves[0].eval(t0)
    nrm = (g1.imag - 1j * g1.real) / np.abs(g1)
    z = np.concatenate([g + h * nrm for h in (1e-4, 1e-3, 1e-2, 0.05, 0.3)])
    tx, ty = z.real, z.imag
    ins = np.zeros(len(tx), np.int8)
    prm = M.make_params(alpha=10.0, tol=TOL, dx=w.dx, batch=2)
    plan = M.Plan(prm, w.boundary, w.volume, (tx, ty, ins), on_surface=True)
    info = plan.info()
    fsrc2 = synth.gauss_source(np.random.default_rng(3), np.array([0.2, -0.3]), np.array([0.1, 0.4]))
    X = np.concatenate([tx, w.boundary["x"]]); Y = np.concatenate([ty, w.boundary["y"]])
    fv = np.stack([w.f_vol, fsrc2(w.volume["x"], w.volume["y"])])
    ft = np.stack([w.meta["fsrc"](X, Y), fsrc2(X, Y)])
    z0 = np.zeros((2, w.n_b))
    out = plan.eval(None, None, _dev(fv), _dev(ft))
    torch.cuda.synchronize()
    V = out[2].cpu().numpy()
    for b in range(2):
        P = O.Problem(10.0, info["delta"], 3, w.boundary, volume=w.volume, targets=(tx, ty), inside=ins,
                      on_surface=True, sigma=z0[b], mu=z0[b], f_vol=fv[b], f_trg=ft[b])
        _, _, Vo = P.eval()
        e = rel_err(V[b], Vo)
        print(f"exterior V batch {b}: err {e:.2e}, finite {np.isfinite(Vo).all()}", flush=True)
        assert np.isfinite(Vo).all()
        assert e < TOL


def test_plan_recreated_reuses_tables(cfg0):
    """A plan created again for the same parameters (a geometry stepped in
    time keeps alpha and delta) takes its level kernel tables from the
    process-wide cache: the same outputs, bit for bit in the level sums and
    the local part."""
    w = cfg0
    print("case plan recreated", flush=True)
    p1 = _plan(w, 7.0)
    a = _run(p1, w, parts=O.PART_LEVELS | O.PART_LOCAL)
    t1 = p1.info()["ms_plan"]
    p1.close()
    p2 = _plan(w, 7.0)
    b = _run(p2, w, parts=O.PART_LEVELS | O.PART_LOCAL)
    t2 = p2.info()["ms_plan"]
    print(f"level phase of plan creation: first {t1[2]:.1f} ms, again {t2[2]:.1f} ms", flush=True)
    for x, y in zip(a, b):
        assert np.array_equal(np.nan_to_num(x, nan=1e300), np.nan_to_num(y, nan=1e300))
