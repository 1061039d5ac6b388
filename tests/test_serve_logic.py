"""Scheduling logic of the request server on the CPU, with a fake device and
a fake clock: admission by memory footprint, LRU eviction of idle plans,
one request per plan at a time, overtaking by other plans, rejection of
requests larger than the budget."""
import numpy as np

from paper_2606_28865_amd.serve import Geometry, Request, Server, latency_stats


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeDevice:
    def __init__(self, clock, plan_bytes, duration):
        self.clock = clock
        self.plan_bytes = plan_bytes        # geometry key -> bytes
        self.duration = duration            # geometry key -> seconds per eval
        self.created, self.destroyed, self.launched = [], [], []
        self.groups, self.inputs, self.batches = [], [], []

    def footprint(self, req, batch=1):
        return self.plan_bytes[req.geometry.key]

    def io_bytes(self, req, batch=1):
        return 10

    def create_plan(self, req, batch=1):
        self.created.append(req.plan_key)
        self.batches.append(batch)
        return {"key": req.plan_key}, self.plan_bytes[req.geometry.key]

    def destroy_plan(self, plan):
        self.destroyed.append(plan["key"])

    def launch(self, plan, group):
        self.launched.extend(r.rid for r in group)
        self.groups.append([r.rid for r in group])
        self.inputs.append([r.u_n for r in group])
        return {"end": self.clock() + self.duration[group[0].geometry.key], "rids": [r.rid for r in group]}

    def done(self, h):
        return self.clock() >= h["end"]

    def result(self, h):
        return [("result", rid) for rid in h["rids"]]


def _geo(key):
    z = np.zeros(16)
    return Geometry(key, {"x": z, "y": z}, None, (np.zeros(0), np.zeros(0), np.zeros(0, np.int8)))


def _req(rid, key, alpha=10.0):
    z = np.zeros(16)
    return Request(rid, _geo(key), alpha, 1e-6, 1, z, z, None, None)


def test_admission_eviction_and_order():
    clk = FakeClock()
    dev = FakeDevice(clk, {"A": 600, "B": 300, "C": 500}, {"A": 1.0, "B": 0.5, "C": 1.0})
    srv = Server(dev, budget_bytes=1000, max_inflight=4, clock=clk)
    for rid, key in enumerate(["A", "A", "B", "C"]):
        srv.submit(_req(rid, key))
    srv.step()
    # A admitted (600+10); second A waits (plan busy); B fits (300+10); C does not fit
    assert dev.launched == [0, 2]
    assert srv.used == 600 + 10 + 300 + 10
    clk.t = 0.6                      # B finishes
    srv.step()
    assert [r.rid for r in srv.finished] == [2]
    assert dev.launched == [0, 2]    # C still needs 510 > 1000 - 610 + 300 idle B -> evict B? B idle now
    # B is idle and evictable: C needs 510, used = 610 + 300 = 910 -> evict B -> 610 + 510 > 1000 -> still waits
    assert "C" not in [k[0] for k in dev.created]
    assert dev.destroyed == []       # evicting B alone would not make room: nothing evicted
    clk.t = 1.0                      # A finishes: second A reuses the resident plan
    srv.step()
    assert dev.launched[2] == 1
    assert dev.created.count(("A", 10.0, 1e-6, 1, "eval")) == 1
    clk.t = 2.0
    srv.step()                       # second A done; C admitted after evicting idle plans
    assert 3 in dev.launched
    assert ("B", 10.0, 1e-6, 1, "eval") in dev.destroyed
    clk.t = 3.5
    srv.step()
    assert sorted(r.rid for r in srv.finished) == [0, 1, 2, 3]
    assert all(r.result == ("result", r.rid) for r in srv.finished)
    st = latency_stats(srv.finished)
    assert st["n"] == 4 and st["p99_ms"] >= st["p50_ms"]


def test_reject_larger_than_budget():
    clk = FakeClock()
    dev = FakeDevice(clk, {"A": 5000}, {"A": 1.0})
    srv = Server(dev, budget_bytes=1000, clock=clk)
    srv.submit(_req(0, "A"))
    srv.step()
    assert len(srv.rejected) == 1 and srv.rejected[0].error
    assert dev.launched == []


def test_run_with_arrivals_overlaps_plans():
    clk = FakeClock()
    dev = FakeDevice(clk, {"A": 100, "B": 100}, {"A": 1.0, "B": 1.0})
    srv = Server(dev, budget_bytes=10_000, clock=clk)
    reqs = [_req(0, "A"), _req(1, "B")]
    reqs[0].arrival = 0.0
    reqs[1].arrival = 0.0
    for r in reqs:
        srv.submit(r)
    srv.step()
    assert sorted(dev.launched) == [0, 1]      # different plans run together
    clk.t = 1.0
    srv.step()
    assert len(srv.finished) == 2


class FailingDevice(FakeDevice):
    """Raises from footprint, create_plan or launch for chosen geometries."""

    def __init__(self, clock, plan_bytes, duration, fail):
        super().__init__(clock, plan_bytes, duration)
        self.fail = fail                     # geometry key -> "footprint" | "create" | "launch"

    def footprint(self, req, batch=1):
        if self.fail.get(req.geometry.key) == "footprint":
            raise RuntimeError("history grid too large")
        return super().footprint(req, batch)

    def create_plan(self, req, batch=1):
        if self.fail.get(req.geometry.key) == "create":
            raise RuntimeError("out of memory")
        return super().create_plan(req, batch)

    def launch(self, plan, group):
        if self.fail.get(group[0].geometry.key) == "launch":
            raise RuntimeError("invalid input")
        return super().launch(plan, group)


def test_failures_are_rejected_and_rolled_back():
    clk = FakeClock()
    dev = FailingDevice(clk, {"A": 100, "F": 100, "C": 100, "L": 100, "B": 100},
                        {"A": 1.0, "F": 1.0, "C": 1.0, "L": 1.0, "B": 1.0},
                        {"F": "footprint", "C": "create", "L": "launch"})
    srv = Server(dev, budget_bytes=10_000, clock=clk)
    for rid, key in enumerate(["F", "A", "C", "L", "B", "L"]):
        srv.submit(_req(rid, key))
    srv.step()
    # every failing request is rejected with its error, the others run
    assert sorted(r.rid for r in srv.rejected) == [0, 2, 3, 5]
    assert all(r.error and r.done >= 0 for r in srv.rejected)
    assert sorted(dev.launched) == [1, 4]
    # the plan whose launch failed stays idle and its bytes are the plan's only
    ent = srv.plans[("L", 10.0, 1e-6, 1, "eval")]
    assert ent["busy"] is False
    assert srv.used == 3 * 100 + 2 * 10          # plans A, L, B; in-flight io of A and B
    assert ("C", 10.0, 1e-6, 1, "eval") not in srv.plans  # creation failed: nothing resident
    assert len(srv.queue) == 0
    clk.t = 1.0
    srv.step()
    assert sorted(r.rid for r in srv.finished) == [1, 4]
    assert srv.used == 3 * 100


def test_failed_completion_query_releases_the_plan():
    clk = FakeClock()
    dev = FakeDevice(clk, {"A": 100}, {"A": 1.0})
    srv = Server(dev, budget_bytes=10_000, clock=clk)
    srv.submit(_req(0, "A"))
    srv.submit(_req(1, "A"))
    srv.step()

    def broken(h):
        raise RuntimeError("device error")
    dev.done = broken
    clk.t = 1.0
    srv.step()
    assert [r.rid for r in srv.rejected] == [0]
    dev.done = lambda h: clk() >= h["end"]
    # the second request was admitted on the released plan in the same pass
    assert dev.launched == [0, 1]
    clk.t = 2.0
    srv.step()
    assert [r.rid for r in srv.finished] == [1]


def test_coalescing_into_the_plan_batch():
    """Queued requests of one plan are launched together, up to the plan's
    batch; a request of another plan is not drawn into the group."""
    clk = FakeClock()
    dev = FakeDevice(clk, {"A": 100, "B": 100}, {"A": 1.0, "B": 1.0})
    srv = Server(dev, budget_bytes=10_000, clock=clk, max_batch=4)
    for rid, key in enumerate(["A", "A", "B", "A", "A", "A", "A"]):
        srv.submit(_req(rid, key))
    assert srv.step() == 5
    assert dev.groups == [[0, 1, 3, 4], [2]]
    assert dev.batches == [4, 4]
    assert [r.rid for r in srv.queue] == [5, 6]
    clk.t = 1.0
    srv.step()
    assert dev.groups[-1] == [5, 6]
    clk.t = 2.0
    srv.step()
    assert sorted(r.rid for r in srv.finished) == list(range(7))
    assert all(r.result == ("result", r.rid) for r in srv.finished)
    assert {r.rid: r.batched_with for r in srv.finished} == {0: 4, 1: 4, 3: 4, 4: 4, 2: 1, 5: 2, 6: 2}


def test_heat_chain_steps_depend_on_each_other():
    """A heat chain's step n + 1 is submitted only when step n has finished,
    with step n's result as its input; two chains overlap."""
    from paper_2606_28865_amd.serve import HeatChain
    clk = FakeClock()
    dev = FakeDevice(clk, {"H1": 100, "H2": 100}, {"H1": 1.0, "H2": 2.0})
    srv = Server(dev, budget_bytes=10_000, clock=clk, max_batch=4)
    chains = [HeatChain(i, _geo(k), 10.0, 1e-10, f"u0-{k}", lambda n: n, 3, rid0=100 * (i + 1))
              for i, k in enumerate(["H1", "H2"])]
    for c in chains:
        srv.submit(c.first())
    srv.step()
    assert dev.groups == [[101], [201]]          # heat steps are never coalesced
    assert dev.inputs == [["u0-H1"], ["u0-H2"]]
    assert dev.batches == [1, 1]
    for t in (1.0, 2.0, 3.0, 4.0, 5.0, 6.0):
        clk.t = t
        srv.step()
    # t = 2: 201 and 102 finish in launch order, so 202 is queued before 103
    assert [g[0] for g in dev.groups] == [101, 201, 102, 202, 103, 203]
    # each step's input is the previous step's result
    assert dev.inputs[2] == ["result"] and dev.inputs[4] == ["result"]
    assert all(c.finished for c in chains)
    assert [s.step for s in chains[0].steps] == [1, 2, 3]
    assert sorted(r.rid for r in srv.finished) == [101, 102, 103, 201, 202, 203]


def test_async_plan_build_keeps_other_plans_running():
    """A new geometry's plan is built in the worker thread: meanwhile the
    loop admits and retires requests of a resident plan; the new plan's
    request runs once the build is done; its footprint is reserved while it
    is built and replaced by the plan's size afterwards; a failed build
    fails the request that waited for it and releases the reservation."""
    import threading
    import time as _time

    clk = FakeClock()
    gate = threading.Event()

    class SlowBuild(FakeDevice):
        def create_plan(self, req, batch=1):
            if req.geometry.key == "B":
                assert gate.wait(10.0)
                if req.alpha == 99.0:
                    raise RuntimeError("build failed")
            return super().create_plan(req, batch)

    dev = SlowBuild(clk, {"A": 100, "B": 200}, {"A": 1.0, "B": 1.0})
    srv = Server(dev, budget_bytes=1000, max_inflight=4, clock=clk, async_build=True)
    srv.submit(_req(0, "A"))
    for _ in range(200):                       # A's plan built in the worker thread
        srv.step()
        if dev.launched == [0]:
            break
        _time.sleep(0.005)
    assert dev.launched == [0]
    srv.submit(_req(1, "B"))
    srv.step()                                 # B's build starts and blocks
    assert srv.used == 100 + 10 + 200          # A resident + its io, B reserved
    clk.t = 1.0
    srv.submit(_req(2, "A"))
    srv.step()                                 # A's first request retires, the second runs, B still building
    assert [r.rid for r in srv.finished] == [0]
    assert dev.launched == [0, 2]
    gate.set()
    for _ in range(200):
        srv.step()
        if 1 in dev.launched:
            break
        _time.sleep(0.005)
    assert dev.launched == [0, 2, 1]
    assert srv.used == 100 + 10 + 200 + 10
    # a failing build: its waiting request is rejected, the reservation released
    clk.t = 2.0
    srv.step()
    used = srv.used
    srv.submit(_req(3, "B", alpha=99.0))
    for _ in range(200):
        srv.step()
        if srv.rejected:
            break
        _time.sleep(0.005)
    assert [r.rid for r in srv.rejected] == [3] and "build failed" in srv.rejected[0].error
    assert srv.used == used
    srv.close()
