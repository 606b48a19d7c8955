"""Scheduling policy of the server (admission by slot and HBM budget,
resident pooling, FIFO order, failure isolation), driven by a host-only
simulated backend: no device work."""

import pytest

from paper_1307_6720_amd import _lib
from paper_1307_6720_amd.serve import Request, Server, percentile


class SimResident:
    def __init__(self, key, nbytes):
        self.key = key
        self.nbytes = nbytes


class SimBackend:
    """Each request finishes after a number of ticks fixed by its id; a
    request whose model is "bad" is rejected at admission."""

    def __init__(self, max_slots, clock):
        self.max_slots = max_slots
        self.clock = clock
        self.slots = {}
        self.live_bytes = 0
        self.peak_live = 0
        self.acquired = 0
        self.admit_order = []
        self.max_concurrent = 0

    def footprint(self, key):
        (nx, ny, nz), _ = key
        return nx * ny * nz * 100

    def acquire(self, key):
        self.acquired += 1
        r = SimResident(key, self.footprint(key))
        self.live_bytes += r.nbytes
        self.peak_live = max(self.peak_live, self.live_bytes)
        return r

    def free(self, res):
        self.live_bytes -= res.nbytes

    def admit(self, res, req):
        if req.model == "bad":
            raise _lib.MHSError(_lib.ERR_NOT_ELLIPTIC, "xi >= 1")
        slot = min(set(range(self.max_slots)) - set(self.slots))
        self.slots[slot] = [req, 2 + req.id % 3]
        self.admit_order.append(req.id)
        self.max_concurrent = max(self.max_concurrent, len(self.slots))
        return slot

    def step(self):
        self.clock.t += 1e-3
        for s in self.slots.values():
            s[1] -= 1
        return sum(1 for s in self.slots.values() if s[1] > 0)

    def poll(self, slot):
        req, left = self.slots[slot]
        done = left <= 0
        st = _lib.ERR_DIVERGED if req.model == "nan" else 0
        return done, {"status": st, "cycles": 3}, {"status": 0, "cycles": 4}

    def release(self, slot):
        del self.slots[slot]


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-6
        return self.t


def make_requests(n, dims_cycle, gap=0.5e-3, models=None):
    out = []
    for i in range(n):
        d = dims_cycle[i % len(dims_cycle)]
        m = models.get(i, "ok") if models else "ok"
        out.append(Request(id=i, dims=d, model=m, bz0=None, arrival=i * gap))
    return out


def test_all_requests_finish_in_fifo_order_and_pool_is_reused():
    clock = Clock()
    be = SimBackend(4, clock)
    srv = Server(be, hbm_budget=10**12)
    reqs = make_requests(40, [(5, 5, 5), (9, 9, 9), (9, 9, 5)])
    done, stats = srv.run(reqs, clock=clock)
    assert stats["requests"] == 40 and stats["ok"] == 40
    assert be.admit_order == sorted(be.admit_order)
    assert be.max_concurrent <= 4
    # residents are pooled per shape: never more than max_slots of a shape
    assert be.acquired <= 3 * 4
    assert stats["p50_ms"] <= stats["p99_ms"]


def test_budget_limits_resident_memory_and_concurrency():
    clock = Clock()
    be = SimBackend(8, clock)
    fp = be.footprint(((9, 9, 9), None))
    srv = Server(be, hbm_budget=2 * fp + fp // 2)
    reqs = make_requests(20, [(9, 9, 9)], gap=0.0)
    done, stats = srv.run(reqs, clock=clock)
    assert stats["ok"] == 20
    assert be.max_concurrent == 2
    assert be.peak_live <= srv.budget


def test_idle_residents_of_other_shapes_are_evicted():
    clock = Clock()
    be = SimBackend(8, clock)
    big = be.footprint(((9, 9, 9), None))
    srv = Server(be, hbm_budget=big + 10)
    reqs = make_requests(6, [(5, 5, 5), (9, 9, 9)], gap=0.0)
    done, stats = srv.run(reqs, clock=clock)
    assert stats["ok"] == 6
    assert be.peak_live <= srv.budget
    assert be.live_bytes <= srv.budget


def test_oversized_request_is_refused():
    clock = Clock()
    be = SimBackend(2, clock)
    srv = Server(be, hbm_budget=1000)
    with pytest.raises(ValueError):
        srv.run(make_requests(1, [(9, 9, 9)]), clock=clock)


def test_failures_are_isolated():
    clock = Clock()
    be = SimBackend(3, clock)
    srv = Server(be, hbm_budget=10**12)
    reqs = make_requests(9, [(5, 5, 5)], models={2: "bad", 5: "nan"})
    done, stats = srv.run(reqs, clock=clock)
    by_id = {r.id: r for r in done}
    assert len(by_id) == 9
    assert by_id[2].status == _lib.ERR_NOT_ELLIPTIC
    assert by_id[5].status == _lib.ERR_DIVERGED
    assert all(by_id[i].status == 0 for i in by_id if i not in (2, 5))
    assert stats["ok"] == 7


def test_late_arrivals_wait_for_their_time():
    clock = Clock()
    be = SimBackend(4, clock)
    srv = Server(be, hbm_budget=10**12)
    reqs = make_requests(5, [(5, 5, 5)], gap=0.05)
    done, _ = srv.run(reqs, clock=clock)
    for r in done:
        assert r.admitted >= r.arrival
        assert r.finished > r.admitted


def test_percentile():
    assert percentile([3, 1, 2], 0.5) == 2
    assert percentile([1.0, 2.0], 0.99) == pytest.approx(1.99)
    assert percentile([], 0.5) is None
