"""Continuous-batching request loop for potential evaluations (Rothe steps).

A Rothe / elliptic-marching solver (paper, Section 1) asks for S, D and V on
the same geometry with the same alpha at every time step, while several such
simulations, of different geometries, sizes, alpha and tolerances, run side
by side.  The server keeps one resident plan per (geometry, alpha, tol,
precision) -- grids, sorted sources, cell lists and kernel tables stay in
HBM -- and runs each admitted request on its plan's own HIP stream, so that
requests of different plans overlap on the device.  A request is admitted as
soon as

  * its plan is idle (a plan is not re-entrant), and
  * the device bytes it needs (a new plan's footprint from
    mhk_plan_footprint, plus its input and output buffers) fit in the memory
    budget; idle plans are evicted least-recently-used to make room.

Requests that do not fit wait in arrival order behind the first waiting
request of the same plan; requests of other plans may overtake it.  Latency
is measured from arrival to the completion event of the request's work.

The scheduling logic is written against a small device interface so that it
can be driven on the CPU by a fake device in tests (admission, eviction,
queueing, rejection of requests larger than the budget).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Dict, List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class Geometry:
    """Host arrays of one geometry: boundary dict (16-node panels), volume
    dict or None, targets (x, y, inside), on_surface flag."""
    key: str
    boundary: dict
    volume: Optional[dict]
    targets: Tuple[np.ndarray, np.ndarray, np.ndarray]
    on_surface: bool = True

    @property
    def n_out(self):
        return len(self.targets[0]) + (len(self.boundary["x"]) if self.on_surface else 0)


@dataclasses.dataclass
class Request:
    rid: int
    geometry: Geometry
    alpha: float
    tol: float
    prec: int                      # 0 FP64, 1 FP32
    sigma: np.ndarray
    mu: np.ndarray
    f_vol: Optional[np.ndarray]
    f_trg: Optional[np.ndarray]
    arrival: float = 0.0
    dx: float = 0.0                # volume mesh size for the split rule
    # filled by the server
    admitted: float = -1.0
    done: float = -1.0
    result: Any = None
    error: Optional[str] = None

    @property
    def plan_key(self):
        return (self.geometry.key, float(self.alpha), float(self.tol), int(self.prec))


class TorchDevice:
    """The real device: plans of libmhk on their own torch streams."""

    def __init__(self):
        import torch
        from . import _lib as L
        self.torch = torch
        self.L = L

    def footprint(self, req: Request) -> int:
        g = req.geometry
        prm = self.L.make_params(alpha=req.alpha, tol=req.tol, prec=req.prec, dx=req.dx)
        return self.L.footprint(prm, g.boundary, g.volume, g.targets, g.on_surface)

    def io_bytes(self, req: Request) -> int:
        g = req.geometry
        es = 8 if req.prec == 0 else 4
        nv = 0 if g.volume is None else len(g.volume["x"])
        return es * (2 * len(g.boundary["x"]) + nv + g.n_out + 3 * g.n_out)

    def create_plan(self, req: Request):
        torch = self.torch
        g = req.geometry
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            prm = self.L.make_params(alpha=req.alpha, tol=req.tol, prec=req.prec, dx=req.dx)
            plan = self.L.Plan(prm, g.boundary, g.volume, g.targets, on_surface=g.on_surface, stream=stream)
        plan_bytes = plan.info()["device_bytes"]
        return plan, plan_bytes

    def destroy_plan(self, plan):
        plan.close()

    def launch(self, plan, req: Request):
        """Upload the densities and enqueue the evaluation on the plan's
        stream; returns a handle polled by done()."""
        torch = self.torch
        dt = torch.float64 if req.prec == 0 else torch.float32
        s = plan.stream
        with torch.cuda.stream(s):
            up = lambda a: None if a is None else torch.from_numpy(
                np.ascontiguousarray(a, dtype=np.float64 if req.prec == 0 else np.float32)).pin_memory().to(
                "cuda", non_blocking=True)
            sig, mu = up(req.sigma), up(req.mu)
            fv = up(req.f_vol) if req.f_vol is not None else None
            ft = up(req.f_trg) if req.f_vol is not None else None
            out = plan.eval(sig, mu, fv, ft)
            host = [None if o is None else torch.empty(o.shape, dtype=dt, pin_memory=True) for o in out]
            for h, o in zip(host, out):
                if o is not None:
                    h.copy_(o, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, host, (sig, mu, fv, ft, out))

    def done(self, handle) -> bool:
        return handle[0].query()

    def result(self, handle):
        return tuple(None if h is None else h.numpy() for h in handle[1])


class Server:
    def __init__(self, device=None, budget_bytes: Optional[int] = None, max_inflight: int = 8,
                 clock: Callable[[], float] = time.perf_counter):
        self.dev = device if device is not None else TorchDevice()
        if budget_bytes is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(free * 0.8)
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.clock = clock
        self.queue: collections.deque = collections.deque()
        self.plans: "collections.OrderedDict[Tuple, Dict]" = collections.OrderedDict()
        self.inflight: List[Tuple[Request, Any, Tuple]] = []
        self.used = 0
        self.finished: List[Request] = []
        self.rejected: List[Request] = []

    # -- submission -----------------------------------------------------
    def submit(self, req: Request):
        if req.arrival <= 0:
            req.arrival = self.clock()
        self.queue.append(req)

    # -- memory accounting ----------------------------------------------
    def _evict_for(self, need: int, keep) -> bool:
        """Evict idle plans, least recently used first, until need bytes fit;
        evict nothing if even evicting every idle plan would not make room."""
        if self.used + need <= self.budget:
            return True
        idle = sum(e["bytes"] for k, e in self.plans.items() if not e["busy"] and k != keep)
        if self.used - idle + need > self.budget:
            return False
        for key in list(self.plans.keys()):
            if self.used + need <= self.budget:
                break
            ent = self.plans[key]
            if ent["busy"] or key == keep:
                continue
            self.dev.destroy_plan(ent["plan"])
            self.used -= ent["bytes"]
            del self.plans[key]
        return self.used + need <= self.budget

    # -- one scheduling pass ----------------------------------------------
    def _fail(self, req: Request, err: Exception):
        req.error = f"{type(err).__name__}: {err}"
        req.done = self.clock()
        self.rejected.append(req)

    def step(self) -> int:
        """Retire finished requests, admit what fits; returns the number of
        requests admitted in this pass.  A request whose footprint, plan
        creation or launch raises is rejected with its error; the plan's
        state and the memory accounting are rolled back and the other
        requests stay queued."""
        still = []
        for req, h, acct in self.inflight:
            try:
                fin = self.dev.done(h)
                if fin:
                    req.result = self.dev.result(h)
            except Exception as e:          # a failed device call: the request ends with its error
                fin = True
                self._fail(req, e)
            if fin:
                ent = self.plans.get(req.plan_key)
                if ent is not None:
                    ent["busy"] = False
                self.used -= acct[0]
                if req.error is None:
                    req.done = self.clock()
                    self.finished.append(req)
            else:
                still.append((req, h, acct))
        self.inflight = still
        admitted = 0
        blocked_keys = set()
        waiting = collections.deque()
        try:
            while self.queue:
                req = self.queue.popleft()
                key = req.plan_key
                if len(self.inflight) >= self.max_inflight or key in blocked_keys:
                    waiting.append(req)
                    continue
                ent = self.plans.get(key)
                if ent is not None and ent["busy"]:
                    blocked_keys.add(key)
                    waiting.append(req)
                    continue
                try:
                    io = self.dev.io_bytes(req)
                    need = io + (0 if ent is not None else self.dev.footprint(req))
                except Exception as e:
                    self._fail(req, e)
                    continue
                if need > self.budget:
                    req.error = f"request needs {need} bytes, budget is {self.budget}"
                    req.done = self.clock()
                    self.rejected.append(req)
                    continue
                if not self._evict_for(need, key):
                    blocked_keys.add(key)
                    waiting.append(req)
                    continue
                if ent is None:
                    try:
                        plan, pbytes = self.dev.create_plan(req)
                    except Exception as e:
                        self._fail(req, e)
                        continue
                    ent = {"plan": plan, "bytes": pbytes, "busy": False}
                    self.plans[key] = ent
                    self.used += pbytes
                self.plans.move_to_end(key)
                req.admitted = self.clock()
                try:
                    h = self.dev.launch(ent["plan"], req)
                except Exception as e:
                    self._fail(req, e)
                    continue
                ent["busy"] = True
                self.used += io
                self.inflight.append((req, h, (io,)))
                admitted += 1
        finally:
            # requests not looked at yet (an unexpected error above) stay
            # queued behind the ones that wait
            waiting.extend(self.queue)
            self.queue = waiting
        return admitted

    def run(self, arrivals: List[Request], poll_s: float = 0.0002):
        """Feed requests at their arrival times (relative seconds) and run
        until all are finished; returns the finished requests."""
        arrivals = sorted(arrivals, key=lambda r: r.arrival)
        t0 = self.clock()
        i = 0
        while i < len(arrivals) or self.queue or self.inflight:
            now = self.clock() - t0
            while i < len(arrivals) and arrivals[i].arrival <= now:
                r = arrivals[i]
                r.arrival = t0 + r.arrival
                self.queue.append(r)
                i += 1
            n = self.step()
            if n == 0 and (self.inflight or (i < len(arrivals))):
                time.sleep(poll_s)
        return self.finished

    def close(self):
        for ent in self.plans.values():
            self.dev.destroy_plan(ent["plan"])
        self.plans.clear()
        self.used = 0


def latency_stats(reqs: List[Request]):
    lat = np.array([r.done - r.arrival for r in reqs if r.error is None])
    if len(lat) == 0:
        return {}
    return {"n": int(len(lat)), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}
