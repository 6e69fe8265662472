"""Host logic of the serving scheduler (paper_2306_11612_amd.serve) with a
simulated engine: memory admission, arrival order, continuous batching,
latency accounting."""
import numpy as np
import pytest

from paper_2306_11612_amd.serve import Job, Scheduler, percentiles, run_open_loop


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-5          # every look at the clock advances it a little
        return self.t


class FakeEngine:
    """A batch takes `fixed + per_job * len` seconds of simulated time after
    it starts; slots run independently."""

    def __init__(self, clock, n_slots=2, fixed=1e-3, per_job=2e-4, bytes_of=None):
        self.clock, self.n_slots, self.fixed, self.per_job = clock, n_slots, fixed, per_job
        self.bytes_of = bytes_of or (lambda j: 1000 * j.n_bins)
        self.started = []
        self.live = 0
        self.max_live = 0
        self.released = []

    def request_bytes(self, job):
        return self.bytes_of(job)

    def start(self, slot, jobs):
        self.started.append((slot, [j.rid for j in jobs]))
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return {"end": self.clock.t + self.fixed + self.per_job * len(jobs), "done": False}

    def finished(self, h):
        if not h["done"] and self.clock.t >= h["end"]:
            h["done"] = True
            self.live -= 1
        return h["done"]

    def release(self, jobs):
        self.released.extend(j.rid for j in jobs)


def _jobs(n, rate, seed=0, widths=(1024, 1920, 3840)):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    return [Job(i, "v", np.zeros((1, 4), np.float32), int(widths[i % len(widths)]), arrival=float(t[i]))
            for i in range(n)]


def test_fifo_runs_one_at_a_time_in_order():
    clk = FakeClock()
    eng = FakeEngine(clk)
    s = Scheduler(eng, budget_bytes=10**9, policy="fifo")
    res = run_open_loop(s, _jobs(50, 2000.0), clock=clk)
    assert res["requests"] == 50
    assert all(len(b) == 1 for _, b in eng.started)
    assert [b[0] for _, b in eng.started] == list(range(50))
    assert eng.max_live == 1
    assert sorted(eng.released) == list(range(50))


def test_batching_groups_waiting_requests_and_respects_slots():
    clk = FakeClock()
    eng = FakeEngine(clk, n_slots=2)
    s = Scheduler(eng, budget_bytes=10**9, max_batch=8, policy="batch")
    res = run_open_loop(s, _jobs(200, 20000.0), clock=clk)
    assert res["requests"] == 200
    assert max(len(b) for _, b in eng.started) <= 8
    assert res["mean_batch"] > 1.5
    assert eng.max_live <= 2
    order = [r for _, b in eng.started for r in b]
    assert order == list(range(200))          # admission never reorders


def test_memory_budget_is_never_exceeded_and_blocks_in_order():
    clk = FakeClock()
    eng = FakeEngine(clk, n_slots=4, bytes_of=lambda j: j.n_bins)
    budget = 5000                              # at most a few requests in flight
    s = Scheduler(eng, budget_bytes=budget, max_batch=32)
    res = run_open_loop(s, _jobs(100, 50000.0), clock=clk)
    assert res["requests"] == 100
    assert s.peak_used <= budget
    assert s.used == 0
    order = [r for _, b in eng.started for r in b]
    assert order == list(range(100))


def test_oversized_request_is_rejected():
    clk = FakeClock()
    s = Scheduler(FakeEngine(clk), budget_bytes=100)
    with pytest.raises(ValueError):
        s.submit(Job(0, "v", np.zeros((1, 4), np.float32), 1024))


def test_batching_beats_fifo_when_overloaded():
    """Arrivals faster than one-at-a-time service: batching keeps up (a batch
    costs a fixed part once), FIFO latency grows with the queue."""
    def run(policy):
        clk = FakeClock()
        eng = FakeEngine(clk, n_slots=2, fixed=1e-3, per_job=1e-4)
        s = Scheduler(eng, budget_bytes=10**12, max_batch=32, policy=policy)
        return run_open_loop(s, _jobs(300, 3000.0, seed=3), clock=clk)
    b, f = run("batch"), run("fifo")
    assert b["p99_ms"] < f["p99_ms"]
    assert b["p50_ms"] < f["p50_ms"]


def test_percentiles():
    p = percentiles([0.001 * k for k in range(1, 101)])
    assert p["p50_ms"] == pytest.approx(50.0)
    assert p["p99_ms"] == pytest.approx(99.0)
    assert percentiles([])["p50_ms"] is None
