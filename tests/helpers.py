"""Shared helpers of the test-suite: plan construction from a seeded
workload, oracle evaluation and error measures."""
import numpy as np

import oracle as O
import synth


def rel_err(gpu, ref):
    """max |gpu - ref| / max |ref| over entries where the oracle is finite;
    the NaN pattern must match exactly."""
    gpu = np.asarray(gpu).ravel()
    ref = np.asarray(ref).ravel()
    m = np.isfinite(ref)
    assert np.array_equal(m, np.isfinite(gpu)), "NaN pattern differs"
    if not m.any():
        return 0.0
    scale = np.abs(ref[m]).max()
    return float(np.abs(gpu[m] - ref[m]).max() / (scale if scale > 0 else 1.0))


def oracle_eval(w, alpha, delta, J, subset=None, parts=O.PART_ALL, sigma=None, mu=None, f_vol=None, f_trg=None,
                on_surface=True):
    P = O.Problem(alpha, delta, J, w.boundary, volume=w.volume, targets=(w.tx, w.ty), inside=w.inside,
                  on_surface=on_surface, sigma=w.sigma if sigma is None else sigma,
                  mu=w.mu if mu is None else mu, f_vol=w.f_vol if f_vol is None else f_vol,
                  f_trg=w.f_trg if f_trg is None else f_trg, parts=parts)
    return P.eval(subset)


def small_multibody(n_bodies=3, n_boundary=2048, n_volume=40_000, n_targets=6000, cfg=11):
    return synth.multibody(cfg=cfg, n_bodies=n_bodies, n_boundary=n_boundary, n_volume=n_volume,
                           n_targets=n_targets, box=0.6)


def stratified_subset(w, band, n_each=64, seed=5):
    """Target indices in output order: some on-surface nodes, some off-surface
    targets inside the given distance band of a node, some elsewhere."""
    from scipy.spatial import cKDTree
    g = np.random.default_rng(seed)
    nt, nb = w.n_t, w.n_b
    bx, by = w.boundary["x"], w.boundary["y"]
    d, _ = cKDTree(np.column_stack([bx, by])).query(np.column_stack([w.tx, w.ty]))
    near = np.nonzero(d < band)[0]
    far = np.nonzero(d >= band)[0]
    pick = lambda a, n: a if len(a) <= n else g.choice(a, n, replace=False)
    on = nt + pick(np.arange(nb), n_each)
    return np.sort(np.concatenate([pick(near, n_each), pick(far, n_each), on])).astype(np.int64)
