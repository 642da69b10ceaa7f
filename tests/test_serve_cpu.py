"""Scheduling logic of the continuous-batching server on the CPU, with a
test-only executor that models device time deterministically (a virtual
clock): admission by budget and slots, FIFO order, every request advanced
exactly its step count, ledger accounting, latency bookkeeping."""
import pytest

from paper_2007_05218_amd import inputs
from paper_2007_05218_amd.serve import Server


class FakeExecutor:
    """Device model: one iteration costs a fixed overhead plus a cost per
    cell of the active set; timing tokens are virtual device times."""

    def __init__(self, per_cell=1e-9, overhead=1e-4):
        self.t = 0.0
        self.per_cell = per_cell
        self.overhead = overhead
        self.active = []
        self.steps_done = {}
        self.batches = []

    def clock(self):
        return self.t

    def sleep(self, dt):
        self.t += dt

    def bytes_needed(self, req):
        return 2 * 40 * (req.n + 8) ** 3 + 768 * (req.n + 8) ** 3

    def admit(self, req):
        req.handle = {"id": req.id}
        self.steps_done[req.id] = 0

    def release(self, req):
        req.handle = None

    def set_batch(self, reqs):
        self.active = list(reqs)
        self.batches.append(sorted(r.id for r in reqs))

    def step(self):
        assert self.active
        for r in self.active:
            assert r.handle is not None
            self.steps_done[r.id] += 1
        self.t += self.overhead + self.per_cell * sum(r.cells for r in self.active)

    def mark(self):
        return self.t

    def wait(self, tok):
        pass

    def elapsed(self, t0, tok):
        return tok - t0


def _server(ex, **kw):
    return Server(ex, clock=ex.clock, sleep=ex.sleep, **kw)


def test_every_request_completes_with_its_steps():
    ex = FakeExecutor()
    specs = inputs.request_stream(60, rate=200.0, seed=3)
    srv = _server(ex, budget_bytes=50e9, max_active=16)
    done = srv.run(specs)
    assert len(done) == 60
    for r in done:
        assert ex.steps_done[r.id] == r.steps
        assert r.t_done >= r.arrival
        # at least `steps` iterations, each at least the overhead
        assert r.t_done - r.arrival >= r.steps * ex.overhead - 1e-12
    assert srv.ledger == pytest.approx(0.0, abs=1e-3)
    m = srv.metrics()
    assert m["p50_s"] <= m["p99_s"]
    assert m["cell_updates"] == sum(r.n ** 3 * r.steps for r in done)


def test_budget_and_slots_respected():
    ex = FakeExecutor()
    specs = inputs.request_stream(40, rate=1e6, seed=5)  # everyone arrives at once
    need = max(ex.bytes_needed(type("R", (), {"n": s["n"]})) for s in specs)
    budget = 3.5 * need
    srv = _server(ex, budget_bytes=budget, max_active=3)
    srv.run(specs)
    assert srv.peak_ledger <= budget
    assert srv.peak_active <= 3
    assert max(len(b) for b in ex.batches) <= 3


def test_fifo_admission():
    ex = FakeExecutor()
    specs = [{"id": i, "arrival": 0.001 * i, "n": 32, "steps": 10 + (i % 3),
              "family": "kh", "seed": i} for i in range(12)]
    srv = _server(ex, budget_bytes=1e12, max_active=2)
    done = srv.run(specs)
    admits = sorted(done, key=lambda r: r.t_admit)
    assert [r.id for r in admits] == list(range(12))


def test_late_arrival_joins_running_batch():
    # continuous batching: a request arriving mid-run is batched with the
    # running one instead of waiting for it to finish
    ex = FakeExecutor(per_cell=1e-9, overhead=1e-3)
    specs = [{"id": 0, "arrival": 0.0, "n": 64, "steps": 100, "family": "kh", "seed": 1},
             {"id": 1, "arrival": 0.02, "n": 32, "steps": 10, "family": "sod", "seed": 2}]
    srv = _server(ex, budget_bytes=1e12)
    done = srv.run(specs)
    assert [0, 1] in ex.batches
    r0, r1 = done
    assert r1.t_done < r0.t_done


def test_request_larger_than_budget_rejected():
    ex = FakeExecutor()
    specs = [{"id": 0, "arrival": 0.0, "n": 192, "steps": 10, "family": "kh", "seed": 1}]
    with pytest.raises(ValueError):
        _server(ex, budget_bytes=1e6).run(specs)


def test_idle_gap_then_arrival():
    ex = FakeExecutor()
    specs = [{"id": 0, "arrival": 0.0, "n": 16, "steps": 3, "family": "kh", "seed": 1},
             {"id": 1, "arrival": 5.0, "n": 16, "steps": 3, "family": "kh", "seed": 2}]
    srv = _server(ex, budget_bytes=1e12)
    done = srv.run(specs)
    assert done[1].t_done >= 5.0
    assert done[1].t_done - done[1].arrival < 1.0
