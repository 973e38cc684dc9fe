"""CPU tests of the serving scheduler with a fake executor and a fake clock:
admission by memory footprint and slots, fused query launches, grouped job
ticks (small jobs whole, large jobs in arrival order in point ranges), the
one-request-per-launch baseline, failure isolation, and the scheduler's
invariants checked at every tick over seeded random streams (a scheduler
that skips the memory test or overfills a slot fails them)."""
import numpy as np

import pytest

from paper_1206_5278_amd.serve import Executor, Scheduler, ServeRequest


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor(Executor):
    """A launch finishes `latency` fake seconds after it starts; a job tick
    finishes after max(latency, pair evaluations / rate)."""

    def __init__(self, clock, latency=1.0, fail_rid=None, sizes=None, rate=None):
        self.clock, self.latency, self.fail_rid = clock, latency, fail_rid
        self.sizes = sizes or {}
        self.rate = rate
        self.launches = []
        self.ranges = {}

    def footprint(self, r):
        return 100 if r.kind == "job" else 10

    def job_points(self, r):
        return self.sizes.get(r.rid, 1000)

    def round_points(self, r):
        return self.round

    round = 256

    def _h(self, kind, reqs):
        if any(r.rid == self.fail_rid for r in reqs):
            raise RuntimeError("injected launch failure")
        self.launches.append((kind, [r.rid for r in reqs], self.clock()))
        return {"t": self.clock() + self.latency, "reqs": reqs}

    def launch_queries(self, set_id, reqs):
        return self._h("query", reqs)

    def launch_job(self, r):
        return self._h("job", [r])

    def prepare_job(self, r):
        pass

    def launch_job_tick(self, items, lane="large"):
        failed = [(r, "injected launch failure") for r, _, _ in items if r.rid == self.fail_rid]
        ok = [(r, i0, i1) for r, i0, i1 in items if r.rid != self.fail_rid]
        self.launches.append(("tick", [(r.rid, i0, i1) for r, i0, i1 in ok], self.clock(), lane))
        for r, i0, i1 in ok:
            self.ranges.setdefault(r.rid, []).append((i0, i1))
        dur = self.latency
        if self.rate:
            dur = max(dur, sum((i1 - i0) * self.job_points(r) * 256.0 for r, i0, i1 in ok) / self.rate)
        # launches of one lane run one after another on its stream
        end = getattr(self, "lane_end", {})
        end[lane] = max(self.clock(), end.get(lane, 0.0)) + dur
        self.lane_end = end
        return {"t": end[lane], "reqs": [r for r, _, _ in ok], "failed": failed}

    def done(self, h):
        return self.clock() >= h["t"]

    def finish(self, h):
        for r in h["reqs"]:
            r.result = r.rid


def drive(sched, clock, step=0.25, limit=5000):
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


def ticks(ex):
    return [l for l in ex.launches if l[0] == "tick"]


def test_batched_fuses_queries_per_set_and_groups_small_jobs():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    s = Scheduler(ex, hbm_budget=10_000, max_active=64, batched=True, clock=clock)
    s.submit_all(reqs_mixed())
    drive(s, clock)
    q_launches = [l for l in ex.launches if l[0] == "query"]
    assert len(q_launches) == 2  # one fused launch per resident set
    assert sorted(sum((l[1] for l in q_launches), [])) == list(range(6))
    # the three small jobs ride whole in one grouped launch
    assert ticks(ex) == [("tick", [(6, 0, 1000), (7, 0, 1000), (8, 0, 1000)], 0.0, "small")]
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


def test_large_jobs_in_arrival_order_small_jobs_ride_along():
    # tick budget 2e12 pair evaluations at 2e13 per fake second: ~0.1 s ticks
    clock = FakeClock()
    sizes = {0: 200_000, 1: 150_000, 2: 2_000, 3: 60_000}
    ex = FakeExecutor(clock, latency=0.01, sizes=sizes, rate=2e13)
    ex.round = 4096
    s = Scheduler(ex, hbm_budget=10_000, batched=True, clock=clock, tick_pairs=2e12)
    s.submit_all([ServeRequest(0, "job", 0.0), ServeRequest(1, "job", 0.1), ServeRequest(2, "job", 0.2),
                  ServeRequest(3, "job", 0.3)])
    drive(s, clock, step=0.01)
    # every job's ranges cover [0, n) in order, inner boundaries at whole
    # rounds of the device (4096 points here)
    for rid, n in sizes.items():
        rs = ex.ranges[rid]
        assert rs[0][0] == 0 and rs[-1][1] == n
        assert all(a[1] == b[0] and a[1] % 4096 == 0 for a, b in zip(rs, rs[1:]))
    assert len(ex.ranges[0]) > 2  # the first large job was split
    done = {r.rid: r.t_done for r in s.completed}
    # the small job, on its own lane, finishes right after it arrives
    assert done[2] <= 0.2 + 0.02
    assert [l[3] for l in ticks(ex) if any(it[0] == 2 for it in l[1])] == ["small"]
    # large jobs run in arrival order: job 1's first range comes in the
    # launch that issues job 0's last one, or later
    large = [l for l in ticks(ex) if l[3] == "large"]
    first1 = min(k for k, l in enumerate(large) if any(it[0] == 1 for it in l[1]))
    last0 = max(k for k, l in enumerate(large) if any(it[0] == 0 for it in l[1]))
    assert first1 >= last0 and done[0] < done[1] <= done[3]
    assert len(s.completed) == 4 and all(r.error is None for r in s.completed)


def test_admission_by_footprint_and_late_arrivals():
    clock = FakeClock()
    ex = FakeExecutor(clock, latency=2.0)
    s = Scheduler(ex, hbm_budget=250, max_active=64, batched=True, clock=clock)
    jobs = [ServeRequest(i, "job", 0.0) for i in range(4)] + [ServeRequest(9, "job", 1.0)]
    s.submit_all(jobs)
    drive(s, clock)
    start = {}
    for _, its, t, _ in ticks(ex):
        for rid, _, _ in its:
            start.setdefault(rid, t)
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
    start = {its[0][0]: t for _, its, t, _ in ticks(ex)}
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
    starts = sorted(t for _, its, t, _ in ticks(ex) for _ in its)
    assert starts[:2] == [0.0, 0.0] and starts[2] >= 1.0


def test_queries_do_not_wait_for_job_slots():
    # two job slots, both taken by long jobs with two more queued: a query
    # that arrives meanwhile is admitted and launched at once
    clock = FakeClock()
    ex = FakeExecutor(clock, latency=2.0)
    s = Scheduler(ex, hbm_budget=10_000, max_active=2, batched=True, clock=clock)
    s.submit_all([ServeRequest(i, "job", 0.0) for i in range(4)] +
                 [ServeRequest(9, "query", 0.5, set_id=0, xq=np.zeros((2, 1), np.float32))])
    drive(s, clock)
    qstart = [t for kind, rids, t, *_ in ex.launches if kind == "query" and 9 in rids]
    assert qstart == [0.5]
    starts = {}
    for _, its, t, _ in ticks(ex):
        for rid, _, _ in its:
            starts.setdefault(rid, t)
    assert starts[0] == 0.0 and starts[1] == 0.0 and starts[2] >= 2.0 and starts[3] >= 2.0
    assert s.active == 0 and s.active_kind == {"job": 0, "query": 0}


def test_memory_is_granted_in_arrival_order():
    # job 1 waits for memory: the younger query does not take memory before
    # it (no starvation of large requests by a stream of small ones)
    clock = FakeClock()
    ex = FakeExecutor(clock, latency=2.0)
    s = Scheduler(ex, hbm_budget=150, max_active=64, batched=True, clock=clock)
    s.submit_all([ServeRequest(0, "job", 0.0), ServeRequest(1, "job", 0.0),
                  ServeRequest(9, "query", 0.25, set_id=0, xq=np.zeros((2, 1), np.float32))])
    drive(s, clock)
    start1 = min(t for _, its, t, _ in ticks(ex) if any(it[0] == 1 for it in its))
    qstart = [t for kind, rids, t, *_ in ex.launches if kind == "query"][0]
    assert start1 >= 2.0 and qstart >= start1
    assert len(s.completed) == 3 and all(r.error is None for r in s.completed)


@pytest.mark.parametrize("batched", [True, False])
def test_failed_launch_fails_only_its_request(batched):
    clock = FakeClock()
    ex = FakeExecutor(clock, fail_rid=7)
    s = Scheduler(ex, hbm_budget=10_000, batched=batched, clock=clock)
    s.submit_all(reqs_mixed())
    drive(s, clock)
    bad = [r for r in s.completed if r.error]
    assert [r.rid for r in bad] == [7]
    assert sum(1 for r in s.completed if r.error is None) == 8
    rep = s.report(1.0)
    assert rep["failed"] == 1 and rep["completed"] == 8 and rep["unfinished"] == 0
    assert s.active == 0 and s.active_kind == {"job": 0, "query": 0} and s.used == 0


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


def _random_stream(seed):
    """Seeded mixed stream: jobs of log-uniform size (small and large, some
    with a failing launch), queries of 1..40 rows on 3 sets, arrivals over
    5 fake seconds."""
    rng = np.random.default_rng(seed)
    reqs, sizes = [], {}
    for rid in range(int(rng.integers(20, 60))):
        t = float(rng.uniform(0.0, 5.0))
        if rng.random() < 0.4:
            reqs.append(ServeRequest(rid, "job", t))
            sizes[rid] = int(np.exp(rng.uniform(np.log(300), np.log(300_000))))
        else:
            reqs.append(ServeRequest(rid, "query", t, set_id=int(rng.integers(0, 3)),
                                     xq=np.zeros((int(rng.integers(1, 41)), 1), np.float32)))
    return reqs, sizes


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("batched", [True, False])
def test_random_streams_keep_the_scheduler_invariants(seed, batched):
    # At every tick: memory in use within the budget, slots within the limit
    # (batched) or one request in service (plain).  At the end: every request
    # finished exactly once, failures only for the failing job, nothing held,
    # each kind admitted in arrival order, and every job's ranges covering
    # [0, n) in order.
    reqs, sizes = _random_stream(seed)
    jobs = [r.rid for r in reqs if r.kind == "job"]
    fail = jobs[len(jobs) // 2] if jobs else None
    clock = FakeClock()
    ex = FakeExecutor(clock, latency=0.05, fail_rid=fail, sizes=sizes, rate=2e12)
    ex.round = 1024
    s = Scheduler(ex, hbm_budget=230, max_active=3, batched=batched, clock=clock, tick_pairs=5e10,
                  small_job_points=4096)
    s.submit_all(reqs)
    s.t0 = clock()
    for _ in range(200_000):
        more = s.tick()
        assert 0 <= s.used <= s.budget
        if batched:
            assert all(0 <= v <= 3 for v in s.active_kind.values())
        else:
            assert s.active <= 1 and len(s.inflight) <= 1
        if not more:
            break
        clock.t += 0.01
    else:
        raise AssertionError("scheduler did not finish")
    assert sorted(r.rid for r in s.completed) == sorted(r.rid for r in reqs)
    assert not s.rejected
    assert {r.rid for r in s.completed if r.error} == ({fail} if fail is not None else set())
    assert all(r.result == r.rid for r in s.completed if r.error is None)
    assert s.used == 0 and s.active == 0 and s.active_kind == {"job": 0, "query": 0}
    rep = s.report(1.0)
    assert rep["unfinished"] == 0 and rep["completed"] + rep["failed"] == len(reqs)
    for kind in ("job", "query"):
        ks = sorted((r for r in reqs if r.kind == kind), key=lambda r: (r.t_arrive, r.rid))
        admits = [r.t_admit for r in ks]
        assert admits == sorted(admits), kind
    if batched:
        for rid, n in sizes.items():
            if rid == fail:
                continue
            rs = ex.ranges[rid]
            assert rs[0][0] == 0 and rs[-1][1] == n
            assert all(a[1] == b[0] for a, b in zip(rs, rs[1:]))
