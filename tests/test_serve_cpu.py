"""CPU tests of the serving scheduler with a fake executor and a fake clock:
admission by memory footprint and slots, FIFO order, fused query launches,
the one-request-per-launch baseline, and failure isolation."""
import numpy as np

import pytest

from paper_1206_5278_amd.serve import Executor, Scheduler, ServeRequest


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor(Executor):
    """Each launch finishes `latency` fake seconds after it starts."""

    def __init__(self, clock, latency=1.0, fail_rid=None):
        self.clock, self.latency, self.fail_rid = clock, latency, fail_rid
        self.launches = []

    def footprint(self, r):
        return 100 if r.kind == "job" else 10

    def _h(self, kind, reqs):
        if any(r.rid == self.fail_rid for r in reqs):
            raise RuntimeError("injected launch failure")
        self.launches.append((kind, [r.rid for r in reqs], self.clock()))
        return {"t": self.clock() + self.latency, "reqs": reqs}

    def launch_queries(self, set_id, reqs):
        return self._h("query", reqs)

    def launch_job(self, r):
        return self._h("job", [r])

    def done(self, h):
        return self.clock() >= h["t"]

    def finish(self, h):
        for r in h["reqs"]:
            r.result = r.rid


def drive(sched, clock, step=0.25, limit=1000):
    sched.t0 = clock()
    for _ in range(limit):
        if not sched.tick():
            return
        clock.t += step
    raise AssertionError("scheduler did not finish")


def reqs_mixed():
    out = []
    for i in range(6):
        out.append(ServeRequest(i, "query", 0.0, set_id=i % 2, xq=np.zeros((3, 1), np.float32)))
    for i in range(6, 9):
        out.append(ServeRequest(i, "job", 0.0))
    return out


def test_batched_fuses_queries_per_set_and_overlaps_jobs():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    s = Scheduler(ex, hbm_budget=10_000, max_active=64, batched=True, clock=clock)
    s.submit_all(reqs_mixed())
    drive(s, clock)
    q_launches = [l for l in ex.launches if l[0] == "query"]
    assert len(q_launches) == 2  # one fused launch per resident set
    assert sorted(sum((l[1] for l in q_launches), [])) == list(range(6))
    assert all(l[2] == 0.0 for l in ex.launches)  # everything started in the first tick
    assert len(s.completed) == 9 and all(r.result == r.rid for r in s.completed)
    assert max(r.latency for r in s.completed) <= 1.25


def test_plain_mode_is_one_request_per_launch_in_order():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    s = Scheduler(ex, hbm_budget=10_000, batched=False, clock=clock)
    s.submit_all(reqs_mixed())
    drive(s, clock)
    assert [l[1] for l in ex.launches] == [[i] for i in range(9)]
    starts = [l[2] for l in ex.launches]
    assert all(b >= a + 1.0 for a, b in zip(starts, starts[1:]))


def test_admission_by_footprint_and_late_arrivals():
    clock = FakeClock()
    ex = FakeExecutor(clock, latency=2.0)
    s = Scheduler(ex, hbm_budget=250, max_active=64, batched=True, clock=clock)
    jobs = [ServeRequest(i, "job", 0.0) for i in range(4)] + [ServeRequest(9, "job", 1.0)]
    s.submit_all(jobs)
    drive(s, clock)
    start = {l[1][0]: l[2] for l in ex.launches}
    assert start[0] == 0.0 and start[1] == 0.0  # two fit in 250 bytes
    assert start[2] >= 2.0 and start[3] >= 2.0  # admitted as memory frees up
    assert start[9] >= 2.0
    assert s.used == 0 and s.active == 0


def test_resident_memory_is_taken_from_the_budget():
    # resident sets hold 100 of 250 bytes: only one 100-byte job fits at a time
    clock = FakeClock()
    ex = FakeExecutor(clock, latency=2.0)
    ex.resident_bytes = lambda: 100
    s = Scheduler(ex, hbm_budget=250, max_active=64, batched=True, clock=clock)
    assert s.budget == 150
    s.submit_all([ServeRequest(i, "job", 0.0) for i in range(2)])
    drive(s, clock)
    start = {l[1][0]: l[2] for l in ex.launches}
    assert start[0] == 0.0 and start[1] >= 2.0
    ex.resident_bytes = lambda: 300
    with pytest.raises(ValueError):
        Scheduler(ex, hbm_budget=250, batched=True, clock=clock)


def test_slot_limit_and_rejection():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    s = Scheduler(ex, hbm_budget=1000, max_active=2, batched=True, clock=clock)
    big = ServeRequest(50, "job", 0.0)
    s.submit_all([ServeRequest(i, "job", 0.0) for i in range(4)])
    ex.footprint = lambda r: 5000 if r.rid == 50 else 100
    s.submit_all([big])
    drive(s, clock)
    assert [r.rid for r in s.rejected] == [50]
    starts = sorted(l[2] for l in ex.launches)
    assert starts[:2] == [0.0, 0.0] and starts[2] >= 1.0


def test_failed_launch_fails_only_its_request():
    clock = FakeClock()
    ex = FakeExecutor(clock, fail_rid=7)
    s = Scheduler(ex, hbm_budget=10_000, batched=True, clock=clock)
    s.submit_all(reqs_mixed())
    drive(s, clock)
    bad = [r for r in s.completed if r.error]
    assert [r.rid for r in bad] == [7]
    assert sum(1 for r in s.completed if r.error is None) == 8
    rep = s.report(1.0)
    assert rep["failed"] == 1 and rep["completed"] == 8


def test_queries_arriving_during_a_batch_join_the_next_batch():
    clock = FakeClock()
    ex = FakeExecutor(clock, latency=1.0)
    s = Scheduler(ex, hbm_budget=10_000, batched=True, clock=clock)
    arrivals = [0.0, 0.25, 0.5, 0.75, 1.0, 3.0]
    s.submit_all([ServeRequest(i, "query", t, set_id=0, xq=np.zeros((2, 1), np.float32))
                  for i, t in enumerate(arrivals)])
    drive(s, clock)
    batches = [l[1] for l in ex.launches]
    # first batch: the query present at t=0; the ones that arrive while it
    # runs are fused into one launch when it completes; the late one alone
    assert batches[0] == [0]
    assert batches[1] == [1, 2, 3, 4]
    assert batches[2] == [5]
