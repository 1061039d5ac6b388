"""Implicit-Euler heat steps (elliptic marching, Section 1) on the device
against the oracle: several steps of the same state, the one-step closed form,
the rejection of plans whose targets are not the volume nodes, and a
full-size step of the 10-body workload checked at sampled nodes (the
oracle's representation V + D[mu] from the device's mu) and by the GMRES
residual.  Bar: 1e-10 relative max-norm, as for the evaluation."""
import numpy as np
import pytest

import oracle as O
import synth
from helpers import rel_err
from oracle import bie

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K = np.pi


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _u0(x, y):
    return np.sin(K * (x + 0.3)) * np.sin(K * (y + 0.2))


def _small():
    cv = synth.Curve(r0=0.5, a=0.1, l1=3)
    b = synth.discretize([cv], 24)
    vol = synth.polar_volume(cv, 24, 96)
    return b, vol


def _plan(b, vol, alpha, delta, on_surface=True, targets=None):
    import paper_2606_28865_amd as M
    tx, ty = (vol["x"], vol["y"]) if targets is None else targets
    return M.Plan(M.make_params(alpha=alpha, tol=1e-10, delta=delta), b, vol, (tx, ty, np.ones(len(tx), np.int8)),
                  on_surface=on_surface)


def test_heat_steps_vs_oracle():
    import paper_2606_28865_amd as M
    b, vol = _small()
    alpha, delta = 3.0, 2e-3
    print("case heat 3 steps small star", flush=True)
    plan = _plan(b, vol, alpha, delta)
    nys = M.Nystrom(alpha, b)
    X = np.concatenate([vol["x"], b["x"]])
    Y = np.concatenate([vol["y"], b["y"]])
    c = alpha ** 2 / (alpha ** 2 + 2 * K * K)
    u_gpu = _dev(_u0(X, Y))
    u_ora = _u0(X, Y)
    for n in range(1, 4):
        g = c ** n * _u0(b["x"], b["y"])
        u_gpu, mu, info = M.heat_step(plan, nys, u_gpu, _dev(g), tol=1e-13)
        _, u_ora = bie.heat_step(alpha, delta, 3, b, vol, u_ora, g)
        e = rel_err(u_gpu.cpu().numpy(), u_ora)
        ex = np.abs(u_ora - c ** n * _u0(X, Y)).max() / np.abs(c ** n * _u0(X, Y)).max()
        print(f"heat step {n}: gpu vs oracle {e:.2e}, oracle vs closed form {ex:.2e}, {info}", flush=True)
        assert info["converged"] == 1
        assert e < 1e-10
    plan.close()
    nys.close()


def test_heat_step_source_term():
    """F^{n+1} enters the source as alpha^2 u^n + F."""
    import paper_2606_28865_amd as M
    b, vol = _small()
    alpha, delta = 5.0, 2e-3
    print("case heat step with F", flush=True)
    plan = _plan(b, vol, alpha, delta)
    nys = M.Nystrom(alpha, b)
    X = np.concatenate([vol["x"], b["x"]])
    Y = np.concatenate([vol["y"], b["y"]])
    u0 = _u0(X, Y)
    F = np.cos(2 * X) * (1 + Y)
    g = 0.5 * _u0(b["x"], b["y"])
    u1, _, info = M.heat_step(plan, nys, _dev(u0), _dev(g), F=_dev(F), tol=1e-13)
    _, ref = bie.heat_step(alpha, delta, 3, b, vol, u0, g, F)
    e = rel_err(u1.cpu().numpy(), ref)
    print(f"heat step with F: err {e:.2e} {info}", flush=True)
    assert e < 1e-10
    plan.close()
    nys.close()


def test_heat_step_rejects_other_targets():
    import paper_2606_28865_amd as M
    b, vol = _small()
    nys = M.Nystrom(3.0, b)
    other = _plan(b, vol, 3.0, 2e-3, targets=(vol["x"][::-1].copy(), vol["y"][::-1].copy()))
    nout = other.n_out
    with pytest.raises(M.MhkError):
        M.heat_step(other, nys, _dev(np.zeros(nout)), _dev(np.zeros(len(b["x"]))))
    other.close()
    nys.close()


def test_heat_step_full_size_sampled():
    """10 bodies, 16384 boundary nodes, ~1M volume nodes as targets, alpha =
    10 (time step 0.01): one step from u0; the device's u at sampled outputs
    against the oracle's V[f] + D[mu] with the device's mu, the interior limit
    on sampled boundary nodes, and the GMRES residual."""
    import paper_2606_28865_amd as M
    from scipy.spatial import cKDTree
    w = synth.multibody(n_targets=10)
    vol = w.volume
    alpha = 10.0
    print(f"case heat full size nv={len(vol['x'])}", flush=True)
    plan = M.Plan(M.make_params(alpha=alpha, tol=1e-10, dx=w.dx), w.boundary, vol,
                  (vol["x"], vol["y"], np.ones(len(vol["x"]), np.int8)), on_surface=True)
    info = plan.info()
    nys = M.Nystrom(alpha, w.boundary)
    X = np.concatenate([vol["x"], w.boundary["x"]])
    Y = np.concatenate([vol["y"], w.boundary["y"]])
    u0 = _u0(X, Y)
    c = alpha ** 2 / (alpha ** 2 + 2 * K * K)
    g = c * _u0(w.boundary["x"], w.boundary["y"])
    u1, mu, sinfo = M.heat_step(plan, nys, _dev(u0), _dev(g), tol=1e-12)
    torch.cuda.synchronize()
    assert sinfo["converged"] == 1 and sinfo["resid"] <= 1e-12
    u1, mu = u1.cpu().numpy(), mu.cpu().numpy()
    nv, nb = len(vol["x"]), w.n_b
    gsel = np.random.default_rng(11)
    d, _ = cKDTree(np.column_stack([w.boundary["x"], w.boundary["y"]])).query(np.column_stack([vol["x"], vol["y"]]))
    near = np.nonzero(d < info["band_volume"])[0]
    far = np.nonzero(d >= info["band_volume"])[0]
    sub = np.sort(np.concatenate([gsel.choice(near, 8, replace=False), gsel.choice(far, 8, replace=False),
                                  nv + gsel.choice(nb, 8, replace=False)])).astype(np.int64)
    f = alpha ** 2 * u0
    P = O.Problem(alpha, info["delta"], 3, w.boundary, volume=vol, targets=(vol["x"], vol["y"]),
                  inside=np.ones(nv, np.int8), on_surface=True, sigma=np.zeros(nb), mu=mu, f_vol=f[:nv], f_trg=f)
    _, D, V = P.eval(sub)
    ref = V + D
    onb = sub >= nv
    ref[onb] -= 0.5 * mu[sub[onb] - nv]
    e = rel_err(u1[sub], ref)
    print(f"heat full size: sampled err {e:.2e}, {sinfo}", flush=True)
    assert e < 1e-10
    plan.close()
    nys.close()
