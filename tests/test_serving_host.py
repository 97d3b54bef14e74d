"""Host-side checks of the serving loop (no GPU): request mix, arrivals, the FIFO
baseline schedule and the continuous-batching scheduler driven by a stand-in executor."""
import math

import numpy as np
import pytest

from paper_1904_02929_amd import serve


def test_mixed_jobs_ranges():
    jobs = serve.mixed_jobs(64, seed=1904, steps=3000, period=1000, u_max=0.05)
    assert len(jobs) == 64
    two = [j for j in jobs if j.kind == "2d"]
    three = [j for j in jobs if j.kind == "3d"]
    assert len(two) == len(three) == 32
    for j in two:
        assert j.L in range(128, 385, 32) and 0.70 <= j.phi <= 0.80 and 0 <= j.theta <= math.pi
        # Lees-Edwards velocity amplitude L * omega * g0 stays below 0.05
        assert j.L * 2 * math.pi / j.period * j.g0 <= 0.05 + 1e-12
    for j in three:
        assert j.L in range(64, 129, 16) and 0.50 <= j.phi <= 0.56
        assert 1e-5 <= j.gamma_dot <= 1e-3 and j.L * j.gamma_dot <= 0.05 + 1e-12
    # reproducible
    again = serve.mixed_jobs(64, seed=1904, steps=3000, period=1000, u_max=0.05)
    assert [(j.L, j.phi, j.seed) for j in jobs] == [(j.L, j.phi, j.seed) for j in again]


def test_poisson_arrivals():
    a = serve.poisson_arrivals(20000, rate=4.0, seed=7)
    assert a[0] == 0.0 and np.all(np.diff(a) >= 0)
    assert abs(np.diff(a).mean() - 0.25) < 0.01


def test_fifo_schedule_by_hand():
    arr = np.array([0.0, 1.0, 1.5, 10.0])
    svc = np.array([2.0, 2.0, 1.0, 1.0])
    fin = serve.fifo_schedule(arr, svc)
    assert fin.tolist() == [2.0, 4.0, 5.0, 11.0]


def test_percentile():
    assert serve.percentile(range(101), 50) == 50.0
    assert serve.percentile(range(101), 99) == 99.0


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExecutor:
    """Footprint = L; the active jobs share a device whose total throughput grows as
    sqrt(number of active jobs) steps per time unit, so that batching pays."""

    def __init__(self, budget, clock):
        self.budget = budget
        self.used = 0
        self.left = {}     # slot -> steps still to run
        self.jobs = {}
        self.clock = clock
        self.last = 0.0
        self.peak = 0
        self.order = []
        self.next = 0

    def _advance(self):
        dt = self.clock() - self.last
        self.last = self.clock()
        run = [s for s, v in self.left.items() if v > 0]
        if run and dt > 0:
            rate = math.sqrt(len(run)) / len(run)
            for s in run:
                self.left[s] -= dt * rate

    def footprint(self, j):
        return j.L

    def add(self, j):
        self._advance()
        if self.used + j.L > self.budget:
            return None
        slot = self.next
        self.next += 1
        self.jobs[slot] = j
        self.used += j.L
        self.order.append(j.jid)
        self.peak = max(self.peak, self.used)
        return slot

    def launch(self, slot, n):
        self._advance()
        self.left[slot] = float(n)

    def poll(self, slot):
        self._advance()
        return self.left[slot] <= 1e-9, 0

    def result(self, slot):
        return self.jobs[slot].jid

    def remove(self, slot):
        self._advance()
        self.used -= self.jobs.pop(slot).L
        self.left.pop(slot)


def test_server_fifo_admission_and_budget():
    jobs = serve.mixed_jobs(16, seed=3, steps=1000)
    arr = serve.poisson_arrivals(16, rate=0.01, seed=4)
    for j, a in zip(jobs, arr):
        j.arrival = float(a)
    clock = Clock()
    ex = FakeExecutor(budget=700, clock=clock)
    srv = serve.Server(ex, budget=700, poll_s=1.0, clock=clock, sleep=clock.sleep)
    done = srv.run(jobs)
    assert sorted(d.jid for d in done) == list(range(16))
    assert ex.peak <= 700 and ex.used == 0
    # admission is first come first served
    by_arrival = [j.jid for j in sorted(jobs, key=lambda j: j.arrival)]
    assert ex.order == by_arrival
    for d in done:
        assert d.result == d.jid
        assert d.arrival <= d.admitted <= d.finished
        assert d.finished - d.admitted >= 1000.0 - 1e-9  # at least its own steps
    # more than one job in flight at some point
    assert max(n for _, n in srv.log) > 1


def test_server_rejects_job_larger_than_budget():
    jobs = serve.mixed_jobs(2, seed=3, steps=10)
    clock = Clock()
    ex = FakeExecutor(budget=50, clock=clock)
    with pytest.raises(ValueError):
        serve.Server(ex, budget=50, clock=clock, sleep=clock.sleep).run(jobs)


def test_server_waits_for_the_head_of_the_queue():
    # budget for one job at a time: jobs finish in arrival order, one after the other
    jobs = serve.mixed_jobs(6, seed=5, steps=100)
    for k, j in enumerate(jobs):
        j.arrival = 0.0
    clock = Clock()
    big = max(j.L for j in jobs)
    ex = FakeExecutor(budget=big, clock=clock)
    done = serve.Server(ex, budget=big, poll_s=0.5, clock=clock, sleep=clock.sleep).run(jobs)
    order = [d.jid for d in sorted(done, key=lambda d: d.finished)]
    assert order == [j.jid for j in jobs]


class FailingExecutor(FakeExecutor):
    """Job `bad` reports an unstable state when its first run completes."""

    def __init__(self, budget, clock, bad):
        super().__init__(budget, clock)
        self.bad = bad

    def poll(self, slot):
        ok, _ = super().poll(slot)
        return ok, (-4 if ok and self.jobs[slot].jid == self.bad else 0)


def test_server_evicts_only_the_failed_job():
    jobs = serve.mixed_jobs(8, seed=7, steps=500)
    for j in jobs:
        j.arrival = 0.0
    clock = Clock()
    ex = FailingExecutor(budget=10 ** 6, clock=clock, bad=3)
    srv = serve.Server(ex, budget=10 ** 6, chunk=100, poll_s=1.0, clock=clock, sleep=clock.sleep)
    done = srv.run(jobs)
    assert sorted(d.jid for d in done) == list(range(8))
    bad = [d for d in done if d.jid == 3][0]
    assert bad.status == -4 and bad.result is None
    # evicted after its first run of 100 steps, long before the others finish
    assert bad.finished - bad.admitted < 0.5 * min(d.finished - d.admitted for d in done if d.jid != 3)
    for d in done:
        if d.jid != 3:
            assert d.status == 0 and d.result == d.jid
    assert ex.used == 0


class FakeLockstepExecutor(FakeExecutor):
    """launch_all(n) runs every admitted job for n steps; records each run's jobs."""

    def __init__(self, budget, clock, bad=None):
        super().__init__(budget, clock)
        self.runs = []
        self.bad = bad

    def launch_all(self, n):
        self._advance()
        assert all(v <= 1e-9 for v in self.left.values()), "a run started before the last ended"
        for s in self.jobs:
            self.left[s] = float(n)
        self.runs.append((sorted(self.jobs), n))

    def poll(self, slot):
        ok, _ = super().poll(slot)
        return ok, (-4 if ok and self.jobs[slot].jid == self.bad else 0)


def test_lockstep_server_runs_every_admitted_job():
    jobs = serve.mixed_jobs(16, seed=3, steps=1000)
    arr = serve.poisson_arrivals(16, rate=0.01, seed=4)
    for j, a in zip(jobs, arr):
        j.arrival = float(a)
    clock = Clock()
    ex = FakeLockstepExecutor(budget=700, clock=clock)
    srv = serve.LockstepServer(ex, budget=700, poll_s=1.0, clock=clock, sleep=clock.sleep)
    done = srv.run(jobs)
    assert sorted(d.jid for d in done) == list(range(16))
    assert ex.peak <= 700 and ex.used == 0
    by_arrival = [j.jid for j in sorted(jobs, key=lambda j: j.arrival)]
    assert ex.order == by_arrival
    # each job took exactly its own steps over the runs it was part of
    slot_of = {}
    for s, j in enumerate(ex.order):
        slot_of[j] = s
    for j in jobs:
        took = sum(n for slots, n in ex.runs if slot_of[j.jid] in slots)
        assert took == j.steps
    for d in done:
        assert d.result == d.jid and d.arrival <= d.admitted <= d.finished
    assert max(len(slots) for slots, _ in ex.runs) > 1


def test_lockstep_server_evicts_only_the_failed_job():
    jobs = serve.mixed_jobs(8, seed=7, steps=500)
    for j in jobs:
        j.arrival = 0.0
    clock = Clock()
    ex = FakeLockstepExecutor(budget=10 ** 6, clock=clock, bad=3)
    srv = serve.LockstepServer(ex, budget=10 ** 6, chunk=100, poll_s=1.0, clock=clock, sleep=clock.sleep)
    done = srv.run(jobs)
    assert sorted(d.jid for d in done) == list(range(8))
    bad = [d for d in done if d.jid == 3][0]
    assert bad.status == -4 and bad.result is None
    for d in done:
        if d.jid != 3:
            assert d.status == 0 and d.result == d.jid
    # the failed job left after the first run; the others ran all their steps
    assert all(ex.order.index(3) not in slots for slots, _ in ex.runs[1:])
    assert ex.used == 0
