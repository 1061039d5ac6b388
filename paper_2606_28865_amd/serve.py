"""Continuous-batching request loop for potential evaluations (Rothe steps).

A Rothe / elliptic-marching solver (paper, Section 1) asks for S, D and V on
the same geometry with the same alpha at every time step, while several such
simulations, of different geometries, sizes, alpha and tolerances, run side
by side.  The server keeps one resident plan per (geometry, alpha, tol,
precision, kind) -- grids, sorted sources, cell lists and kernel tables stay
in HBM -- and runs each admitted request on its plan's own HIP stream, so
that requests of different plans overlap on the device.  A request is
admitted as soon as

  * its plan is idle (a plan is not re-entrant), and
  * the device bytes it needs (a new plan's footprint from
    mhk_plan_footprint, plus its input and output buffers) fit in the memory
    budget; idle plans are evicted least-recently-used to make room.

Requests of one plan that are queued together are coalesced into the
plan's batch dimension (up to max_batch densities per launch: the level
sums share each kernel-table evaluation across them, the closest points and
local coefficients are shared by the batch), so a burst of same-geometry
steps costs one evaluation of the batch.

Two kinds of request: "eval" (S, D, V of given densities) and "heat" (one
implicit-Euler step of the heat equation, a Dirichlet solve with the source
alpha^2 u^n; the plan's targets are the volume nodes).  A heat step's input
is the previous step's result, so a simulation is a chain: the server calls
the request's on_done, which may return the next step (HeatChain below).
Heat steps run their blocking GMRES solve in a worker thread each (the
library call releases the interpreter), so that several chains and the eval
requests overlap on the device.

Requests that do not fit wait in arrival order behind the first waiting
request of the same plan; requests of other plans may overtake it.  Latency
is measured from arrival to the completion of the request's work.

The scheduling logic is written against a small device interface so that it
can be driven on the CPU by a fake device in tests (admission, eviction,
queueing, coalescing, chains, rejection of requests larger than the budget).
"""
from __future__ import annotations

import collections
import concurrent.futures
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
    sigma: Any = None
    mu: Any = None
    f_vol: Any = None
    f_trg: Any = None
    arrival: float = 0.0
    dx: float = 0.0                # volume mesh size for the split rule
    kind: str = "eval"             # "eval" or "heat"
    u_n: Any = None                # heat: u^n at the volume nodes then the boundary nodes
    g_next: Any = None             # heat: boundary data of the new step
    F: Any = None                  # heat: source of the new step (or None)
    on_done: Optional[Callable[["Request"], Optional["Request"]]] = None
    # filled by the server
    admitted: float = -1.0
    done: float = -1.0
    result: Any = None
    error: Optional[str] = None
    batched_with: int = 1          # requests in the launch that served this one

    @property
    def plan_key(self):
        return (self.geometry.key, float(self.alpha), float(self.tol), int(self.prec), self.kind)

    def pattern(self):
        """Which inputs an eval request carries (requests are coalesced only
        with requests of the same pattern)."""
        return (self.sigma is not None, self.mu is not None, self.f_vol is not None)


class HeatChain:
    """A time-stepping simulation driven through the server: step n + 1 is
    submitted when step n has finished, with u^{n+1} of step n as its u^n
    (kept on the device).  g_of_step(n) gives the boundary data of step n
    (n = 1..nsteps), F_of_step(n) the source (or None)."""

    def __init__(self, sid, geometry, alpha, tol, u0, g_of_step, nsteps, F_of_step=None, dx=0.0, rid0=0):
        self.sid, self.geometry, self.alpha, self.tol = sid, geometry, float(alpha), float(tol)
        self.u0, self.g_of_step, self.F_of_step = u0, g_of_step, F_of_step
        self.nsteps, self.dx, self.rid0 = int(nsteps), dx, rid0
        self.steps: List[Request] = []

    def _req(self, n, u_n, arrival=0.0):
        r = Request(self.rid0 + n, self.geometry, self.alpha, self.tol, 0, arrival=arrival, dx=self.dx, kind="heat",
                    u_n=u_n, g_next=self.g_of_step(n), F=None if self.F_of_step is None else self.F_of_step(n),
                    on_done=self._next)
        r.step = n
        self.steps.append(r)
        return r

    def first(self, arrival=0.0) -> Request:
        return self._req(1, self.u0, arrival)

    def _next(self, req: Request) -> Optional[Request]:
        if req.error is not None or req.step >= self.nsteps:
            return None
        return self._req(req.step + 1, req.result[0])

    @property
    def finished(self):
        return len(self.steps) == self.nsteps and self.steps[-1].done >= 0


class TorchDevice:
    """The real device: plans of libmhk on their own torch streams, on the
    device current when it is constructed (or `device`).  Worker threads
    start on device 0, so every plan's stream is made on that device and
    the work of a plan runs inside its stream's context, which selects it."""

    def __init__(self, workers: int = 4, device: Optional[int] = None):
        import torch
        from . import _lib as L
        self.torch = torch
        self.L = L
        self.index = torch.cuda.current_device() if device is None else int(device)
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=workers)

    def _params(self, req: Request, batch: int):
        return self.L.make_params(alpha=req.alpha, tol=req.tol, prec=req.prec, dx=req.dx, batch=batch)

    def footprint(self, req: Request, batch: int = 1) -> int:
        g = req.geometry
        b = self.L.footprint(self._params(req, batch), g.boundary, g.volume, g.targets, g.on_surface)
        if req.kind == "heat":
            nb = len(g.boundary["x"])
            b += 8 * nb * (nb + 1) + 8 * 70 * nb     # Nystrom matrix and GMRES workspace
        return b

    def io_bytes(self, req: Request, batch: int = 1) -> int:
        g = req.geometry
        es = 8 if req.prec == 0 else 4
        nv = 0 if g.volume is None else len(g.volume["x"])
        if req.kind == "heat":
            return 8 * (4 * g.n_out + 2 * len(g.boundary["x"]))
        return es * batch * (2 * len(g.boundary["x"]) + nv + g.n_out + 3 * g.n_out)

    def create_plan(self, req: Request, batch: int = 1):
        torch = self.torch
        g = req.geometry
        stream = torch.cuda.Stream(device=self.index)
        with torch.cuda.stream(stream):
            plan = self.L.Plan(self._params(req, batch), g.boundary, g.volume, g.targets, on_surface=g.on_surface,
                               stream=stream)
            nbytes = plan.info()["device_bytes"]
            if req.kind == "heat":
                nys = self.L.Nystrom(req.alpha, g.boundary, stream=stream)
                nbytes += nys.info()["device_bytes"]
                return (plan, nys), nbytes
        return plan, nbytes

    def destroy_plan(self, plan):
        if isinstance(plan, tuple):
            plan[1].close()
            plan = plan[0]
        plan.close()

    def _dev(self, a, dt):
        torch = self.torch
        if a is None:
            return None
        if isinstance(a, torch.Tensor):
            return a.to(device="cuda", dtype=dt).contiguous()
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64 if dt == torch.float64 else np.float32)
                                ).pin_memory().to("cuda", non_blocking=True)

    def launch(self, plan, group: List[Request]):
        """Upload the inputs and enqueue the work on the plan's stream (eval:
        the group's densities stacked, evaluated as a batch of that size on
        the plan sized for max_batch; heat: the solve in a worker thread);
        returns a handle polled by done()."""
        torch = self.torch
        if group[0].kind == "heat":
            return self._launch_heat(plan, group[0])
        dt = torch.float64 if group[0].prec == 0 else torch.float32
        s = plan.stream
        G = len(group)
        with torch.cuda.stream(s):
            def stack(name, n):
                if getattr(group[0], name) is None:
                    return None
                h = np.empty((G, n), np.float64 if dt == torch.float64 else np.float32)
                for i, r in enumerate(group):
                    h[i] = np.asarray(getattr(r, name)).ravel()
                return self._dev(h, dt)
            nb, nv, no = plan.nb, plan.nv, plan.n_out
            sig, mu, fv = stack("sigma", nb), stack("mu", nb), stack("f_vol", nv)
            ft = stack("f_trg", plan.f_rows * no) if fv is not None else None
            # the group's densities only: a launch costs what it carries
            out = plan.eval(sig, mu, fv, ft, nbatch=G)
            host = [None if o is None else torch.empty(o.shape, dtype=dt, pin_memory=True) for o in out]
            for h, o in zip(host, out):
                if o is not None:
                    h.copy_(o, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return ("eval", ev, host, len(group), (sig, mu, fv, ft, out))

    def _launch_heat(self, pair, req: Request):
        torch = self.torch
        plan, nys = pair
        with torch.cuda.stream(plan.stream):
            u = self._dev(req.u_n, torch.float64)
            g = self._dev(req.g_next, torch.float64)
            F = self._dev(req.F, torch.float64)
        plan.stream.synchronize()            # uploads done before the worker's solve reads them

        def work():
            with torch.cuda.stream(plan.stream):
                u1, mu, info = self.L.heat_step(plan, nys, u, g, F=F, tol=1e-12)
            return u1, mu, info
        return ("heat", self.pool.submit(work))

    def done(self, handle) -> bool:
        return handle[1].query() if handle[0] == "eval" else handle[1].done()

    def result(self, handle):
        if handle[0] == "heat":
            return [handle[1].result()]
        host, n = handle[2], handle[3]
        return [tuple(None if h is None else h[i].numpy() for h in host) for i in range(n)]

    def close(self):
        self.pool.shutdown(wait=True)


class Server:
    """Request loop over a device (TorchDevice, or a fake one in tests).

    async_build: create new plans in worker threads (default: on for the
    real device; build_workers of them, each plan on its own stream), so
    that the loop keeps retiring and admitting requests of other plans while
    new geometries' plans are built; a request waits behind its plan, whose
    footprint is reserved while it is built."""

    def __init__(self, device=None, budget_bytes: Optional[int] = None, max_inflight: int = 8,
                 clock: Callable[[], float] = time.perf_counter, max_batch: int = 1,
                 async_build: Optional[bool] = None, build_workers: int = 2):
        self.async_build = (device is None) if async_build is None else bool(async_build)
        self.builder = (concurrent.futures.ThreadPoolExecutor(max_workers=max(1, int(build_workers)))
                        if self.async_build else None)
        self.dev = device if device is not None else TorchDevice()
        if budget_bytes is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(free * 0.8)
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.max_batch = max(1, int(max_batch))
        self.clock = clock
        self.queue: collections.deque = collections.deque()
        self.plans: "collections.OrderedDict[Tuple, Dict]" = collections.OrderedDict()
        # in flight: (requests of one launch, handle, io bytes)
        self.inflight: List[Tuple[List[Request], Any, int]] = []
        self.used = 0
        self.finished: List[Request] = []
        self.rejected: List[Request] = []
        self.build_errors: Dict[Tuple, Exception] = {}

    def _batch(self, req: Request) -> int:
        """Batch capacity of the plan a request runs on."""
        return self.max_batch if req.kind == "eval" else 1

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

    def _finish(self, req: Request):
        """Completion of one request: record it and submit what its chain
        asks for next."""
        if req.error is None:
            req.done = self.clock()
            self.finished.append(req)
        if req.on_done is not None:
            nxt = req.on_done(req)
            if nxt is not None:
                self.submit(nxt)

    def _poll_builds(self):
        """Plans built in the worker thread: resident once done (their
        reservation replaced by their actual size), or dropped with the
        error that the next request of the plan will carry."""
        for key, ent in list(self.plans.items()):
            fut = ent.get("building")
            if fut is None or not fut.done():
                continue
            ent["building"] = None
            try:
                plan, pbytes = fut.result()
            except Exception as e:
                self.used -= ent["bytes"]
                del self.plans[key]
                self.build_errors[key] = e
                continue
            self.used += pbytes - ent["bytes"]
            ent.update(plan=plan, bytes=pbytes, busy=False)

    def step(self) -> int:
        """Retire finished launches, admit what fits; returns the number of
        requests admitted in this pass.  A request whose footprint, plan
        creation or launch raises is rejected with its error; the plan's
        state and the memory accounting are rolled back and the other
        requests stay queued."""
        if self.async_build:
            self._poll_builds()
        still = []
        for group, h, io in self.inflight:
            try:
                fin = self.dev.done(h)
                if fin:
                    res = self.dev.result(h)
                    for r, x in zip(group, res):
                        r.result = x
            except Exception as e:          # a failed device call: the requests end with its error
                fin = True
                for r in group:
                    self._fail(r, e)
            if fin:
                ent = self.plans.get(group[0].plan_key)
                if ent is not None:
                    ent["busy"] = False
                self.used -= io
                for r in group:
                    self._finish(r)
            else:
                still.append((group, h, io))
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
                if key in self.build_errors:
                    self._fail(req, self.build_errors.pop(key))
                    continue
                ent = self.plans.get(key)
                if ent is not None and ent["busy"]:
                    blocked_keys.add(key)
                    waiting.append(req)
                    continue
                B = self._batch(req)
                try:
                    io = self.dev.io_bytes(req, B)
                    need = io + (0 if ent is not None else self.dev.footprint(req, B))
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
                if ent is None and self.async_build:
                    # build in the worker thread, the footprint reserved;
                    # the request waits for its plan
                    fp = need - io
                    self.plans[key] = {"plan": None, "bytes": fp, "busy": True,
                                       "building": self.builder.submit(self.dev.create_plan, req, B)}
                    self.used += fp
                    blocked_keys.add(key)
                    waiting.append(req)
                    continue
                if ent is None:
                    try:
                        plan, pbytes = self.dev.create_plan(req, B)
                    except Exception as e:
                        self._fail(req, e)
                        continue
                    ent = {"plan": plan, "bytes": pbytes, "busy": False}
                    self.plans[key] = ent
                    self.used += pbytes
                self.plans.move_to_end(key)
                # coalesce: the queued requests of the same plan and input
                # pattern, in arrival order, up to the plan's batch
                group = [req]
                if B > 1:
                    rest = collections.deque()
                    while self.queue:
                        r = self.queue.popleft()
                        if len(group) < B and r.plan_key == key and r.pattern() == req.pattern():
                            group.append(r)
                        else:
                            rest.append(r)
                    self.queue = rest
                now = self.clock()
                for r in group:
                    r.admitted = now
                    r.batched_with = len(group)
                try:
                    h = self.dev.launch(ent["plan"], group)
                except Exception as e:
                    for r in group:
                        self._fail(r, e)
                    continue
                ent["busy"] = True
                self.used += io
                self.inflight.append((group, h, io))
                admitted += len(group)
        finally:
            # requests not looked at yet (an unexpected error above) stay
            # queued behind the ones that wait
            waiting.extend(self.queue)
            self.queue = waiting
        return admitted

    def run(self, arrivals: List[Request], poll_s: float = 0.0002):
        """Feed requests at their arrival times (relative seconds) and run
        until all are finished, chains included; returns the finished
        requests."""
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
            building = any(e.get("building") is not None for e in self.plans.values())
            if n == 0 and (self.inflight or building or (i < len(arrivals))):
                time.sleep(poll_s)
        return self.finished

    def close(self):
        if self.builder is not None:
            self.builder.shutdown(wait=True)
            self._poll_builds()
        for ent in self.plans.values():
            if ent["plan"] is not None:
                self.dev.destroy_plan(ent["plan"])
        self.plans.clear()
        self.used = 0
        if hasattr(self.dev, "close"):
            self.dev.close()


def latency_stats(reqs: List[Request]):
    lat = np.array([r.done - r.arrival for r in reqs if r.error is None])
    if len(lat) == 0:
        return {}
    return {"n": int(len(lat)), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}
