"""CPU tests of the serving scheduler with a simulated clock and a fake
executor (service time proportional to cells x steps of the chunk)."""
import numpy as np
import pytest

from paper_2310_00236_amd.serve import Job, Scheduler


class FakeExec:
    def __init__(self, clock, rate=1e9):
        self.clock = clock
        self.rate = rate
        self.resident = {}
        self.events = []
        self.pending = 0.0
        self.max_bytes = 0

    def admit(self, job):
        self.resident[job.id] = job
        self.events.append(("admit", job.id, self.clock.t))
        self.max_bytes = max(self.max_bytes, sum(j.footprint for j in self.resident.values()))

    def launch(self, jobs, steps):
        for j in jobs:
            assert j.id in self.resident
        self.pending = sum(j.cells * s for j, s in zip(jobs, steps)) / self.rate
        self.events.append(("launch", tuple(j.id for j in jobs), self.clock.t))

    def wait(self):
        self.clock.t += self.pending
        self.pending = 0.0

    def retire(self, job):
        del self.resident[job.id]
        self.events.append(("retire", job.id, self.clock.t))
        return ("result", job.id)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def _jobs(n, seed=0, rate=5.0):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1 / rate)
        cells = int(rng.integers(1, 50)) * 100000
        out.append(Job(id=i, arrival=t, footprint=cells * 32, nsteps=int(rng.integers(100, 2000)),
                       cells=cells))
    return out


def test_budget_never_exceeded_and_all_complete():
    clk = Clock()
    ex = FakeExec(clk)
    jobs = _jobs(60)
    budget = 80 * 100000 * 32
    s = Scheduler(ex, budget, chunk_steps=100, clock=clk, idle=clk.sleep)
    st = s.run(jobs)
    assert st.rejected == 0
    assert len(s.done) == 60 and all(j.result == ("result", j.id) for j in s.done)
    assert ex.max_bytes <= budget and st.peak_bytes <= budget
    assert all(j.finished >= j.admitted >= j.arrival for j in s.done)
    assert all(j.done_steps == j.nsteps for j in s.done)
    summ = st.summary()
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0
    assert summ["completed"] == 60


def test_admission_is_fifo_and_overlaps_running_work():
    clk = Clock()
    ex = FakeExec(clk)
    jobs = _jobs(40, seed=1, rate=50.0)
    s = Scheduler(ex, 60 * 100000 * 32, chunk_steps=50, clock=clk, idle=clk.sleep)
    s.run(jobs)
    admits = [e[1] for e in ex.events if e[0] == "admit"]
    assert admits == sorted(admits)                 # first come, first served
    # some request was admitted while others were resident (continuous batching)
    launches = [set(e[1]) for e in ex.events if e[0] == "launch"]
    assert any(len(a) > 1 for a in launches)
    joined_late = any(b - a and a & b for a, b in zip(launches, launches[1:]))
    assert joined_late


def test_oversized_request_rejected_not_blocking():
    clk = Clock()
    ex = FakeExec(clk)
    jobs = _jobs(10, seed=2)
    jobs[3].footprint = 10 ** 15
    s = Scheduler(ex, 60 * 100000 * 32, chunk_steps=100, clock=clk, idle=clk.sleep)
    st = s.run(jobs)
    assert st.rejected == 1 and len(s.done) == 9


def test_waits_for_late_arrivals():
    clk = Clock()
    ex = FakeExec(clk)
    jobs = [Job(id=0, arrival=5.0, footprint=10, nsteps=10, cells=10),
            Job(id=1, arrival=100.0, footprint=10, nsteps=10, cells=10)]
    s = Scheduler(ex, 100, chunk_steps=100, clock=clk, idle=clk.sleep)
    st = s.run(jobs)
    assert [j.id for j in s.done] == [0, 1]
    assert s.done[1].admitted >= 100.0
    assert st.summary()["completed"] == 2


def test_bad_parameters():
    with pytest.raises(ValueError):
        Scheduler(None, 0, 10, clock=lambda: 0.0, idle=lambda d: None)
