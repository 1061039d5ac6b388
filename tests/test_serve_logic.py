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

    def footprint(self, req):
        return self.plan_bytes[req.geometry.key]

    def io_bytes(self, req):
        return 10

    def create_plan(self, req):
        self.created.append(req.plan_key)
        return {"key": req.plan_key}, self.plan_bytes[req.geometry.key]

    def destroy_plan(self, plan):
        self.destroyed.append(plan["key"])

    def launch(self, plan, req):
        self.launched.append(req.rid)
        return {"end": self.clock() + self.duration[req.geometry.key], "rid": req.rid}

    def done(self, h):
        return self.clock() >= h["end"]

    def result(self, h):
        return ("result", h["rid"])


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
    assert dev.created.count(("A", 10.0, 1e-6, 1)) == 1
    clk.t = 2.0
    srv.step()                       # second A done; C admitted after evicting idle plans
    assert 3 in dev.launched
    assert ("B", 10.0, 1e-6, 1) in dev.destroyed
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

    def footprint(self, req):
        if self.fail.get(req.geometry.key) == "footprint":
            raise RuntimeError("history grid too large")
        return super().footprint(req)

    def create_plan(self, req):
        if self.fail.get(req.geometry.key) == "create":
            raise RuntimeError("out of memory")
        return super().create_plan(req)

    def launch(self, plan, req):
        if self.fail.get(req.geometry.key) == "launch":
            raise RuntimeError("invalid input")
        return super().launch(plan, req)


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
    ent = srv.plans[("L", 10.0, 1e-6, 1)]
    assert ent["busy"] is False
    assert srv.used == 3 * 100 + 2 * 10          # plans A, L, B; in-flight io of A and B
    assert ("C", 10.0, 1e-6, 1) not in srv.plans  # creation failed: nothing resident
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
