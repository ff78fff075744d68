"""The serving scheduler with a simulated executor and clock (no GPU): admission by arrival,
free slots and the memory budget; first-come first-served; every request finishes."""
import time

import numpy as np
import pytest

from paper_2203_00952_amd.serve import Job, Scheduler, percentile


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Each job runs for `duration(job)` seconds of fake time from the moment it starts."""

    def __init__(self, clock, duration):
        self.clock, self.duration = clock, duration
        self.running = {}
        self.log = []

    def start(self, job, slot):
        end = self.clock() + self.duration(job)
        self.log.append((self.clock(), job.rid, slot))
        self.running[job.rid] = end
        return job.rid

    def done(self, h):
        return self.clock() >= self.running[h]

    def finish_time(self, h, t0):
        return self.running[h] - t0


def _advance(clock, ex):
    def idle(dt):
        # jump to the next completion or arrival, at least a small step
        pending_ends = [e for e in ex.running.values() if e > clock.t]
        step = min(pending_ends) - clock.t if pending_ends else dt
        clock.t += max(min(step, dt) if dt > 0 else step, 1e-6)
    return idle


def run(jobs, slots, budget, duration):
    clock = FakeClock()
    ex = FakeExecutor(clock, duration)
    sch = Scheduler(ex, slots, budget, clock=clock, idle=_advance(clock, ex))
    return sch.run(jobs), ex, sch


def test_all_finish_and_respect_slots_and_budget():
    rng = np.random.default_rng(0)
    arrivals = np.cumsum(rng.exponential(0.01, 200))
    sizes = rng.integers(1, 40, 200) * 100
    jobs = [Job(i, float(a), int(s)) for i, (a, s) in enumerate(zip(arrivals, sizes))]
    recs, ex, sch = run(jobs, slots=3, budget=6000, duration=lambda j: j.nbytes / 1e5)
    assert [r.rid for r in recs] == list(range(200))
    assert sch.peak_bytes <= 6000
    for r in recs:
        assert r.admitted >= r.arrival - 1e-12
        assert r.finished >= r.admitted + jobs[r.rid].nbytes / 1e5 - 1e-9
    # never more than `slots` jobs at once
    events = sorted([(r.admitted, 1) for r in recs] + [(r.finished, -1) for r in recs])
    live = np.cumsum([e[1] for e in events])
    assert live.max() <= 3


def test_first_come_first_served():
    jobs = [Job(0, 0.0, 900), Job(1, 0.001, 900), Job(2, 0.002, 100)]
    recs, ex, _ = run(jobs, slots=4, budget=1000, duration=lambda j: 1.0)
    order = [rid for _, rid, _ in ex.log]
    assert order == [0, 1, 2]                  # job 2 fits beside job 0 but waits behind job 1
    assert recs[2].admitted >= recs[1].admitted


def test_budget_is_binding_and_overlap_happens():
    jobs = [Job(i, 0.0, 400) for i in range(6)]
    recs, _, sch = run(jobs, slots=6, budget=1000, duration=lambda j: 1.0)
    assert sch.peak_bytes == 800                 # two at a time fit
    fins = sorted(r.finished for r in recs)
    assert fins == pytest.approx([1, 1, 2, 2, 3, 3], abs=1e-3)


def test_oversized_request_is_rejected():
    with pytest.raises(ValueError):
        run([Job(0, 0.0, 5000)], slots=1, budget=1000, duration=lambda j: 1.0)


def test_percentile():
    assert percentile([1, 2, 3, 4], 50) == 2.5
    assert percentile([5], 99) == 5


class ThreadExecutor:
    """Jobs complete on timer threads after `duration(job)` seconds of wall time; the executor
    offers token/wait like the GPU one, and counts how often the scheduler polls `done`."""

    def __init__(self, duration):
        import threading

        self.duration = duration
        self.cv = threading.Condition()
        self.completions = 0
        self.polls = 0
        self.ends = {}

    def start(self, job, slot):
        import threading

        def fin():
            with self.cv:
                self.ends[job.rid] = time.perf_counter()
                self.completions += 1
                self.cv.notify_all()

        threading.Timer(self.duration(job), fin).start()
        return job.rid

    def done(self, h):
        with self.cv:
            self.polls += 1
            return h in self.ends

    def finish_time(self, h, t0):
        return self.ends[h] - t0

    def token(self):
        with self.cv:
            return self.completions

    def wait(self, token, timeout):
        with self.cv:
            self.cv.wait_for(lambda: self.completions != token, timeout)


def test_scheduler_sleeps_instead_of_spinning():
    """With an executor that can block, the scheduler waits for completions and arrivals: the
    number of `done` polls stays near (jobs x slots), not proportional to wall time."""
    jobs = [Job(i, 0.004 * i, 100) for i in range(20)]
    ex = ThreadExecutor(lambda j: 0.01)
    sch = Scheduler(ex, slots=2, budget_bytes=1000)
    t0 = time.perf_counter()
    recs = sch.run(jobs)
    wall = time.perf_counter() - t0
    assert [r.rid for r in recs] == list(range(20))
    assert all(r.finished >= r.admitted >= r.arrival - 1e-3 for r in recs)
    assert wall > 0.08                       # 20 jobs of 10 ms on 2 slots
    assert ex.polls < 400, ex.polls          # a spinning loop polls ~1e5 times in 0.1 s
