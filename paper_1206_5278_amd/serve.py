"""Continuous-batching server for bandwidth-selection jobs and conditional
density queries (the estimator of eq. 1 and the criterion of eq. 3).

Two request kinds:
  * job   -- exact LOO log-likelihood over a scalar bandwidth grid on the
             request's own training set (``cde_create`` + ``cde_loo_loglik``);
             the answer is the grid of totals and its argmax.
  * query -- f(y | x) for q query points on a y-grid against one of the
             resident training sets (``cde_density_query``).

Scheduling (one scheduler thread, ``tick`` is one pass):
  1. arrivals whose time has come enter the waiting queue of their kind;
  2. admission: each request kind (job, query) has its own FIFO queue and
     its own slots, so queries never wait for a slot behind queued jobs;
     device memory is granted in arrival order across both queues (the
     oldest request that is free to go and does not fit the HBM budget stops
     all admission until memory frees up, so no request starves).  Requests
     arriving while others run are admitted as slots and memory free up; an
     admitted job's data is uploaded and its model created at once;
  3. launch: admitted queries wait in a per-set ready list; whenever a
     resident set has no query launch in flight, all of its ready queries
     become ONE fused query launch (so queries that arrive while a batch runs
     join the next batch).  Jobs run in grouped launches (``cde_launch_batch``)
     of work items, each item a range of one job's points, on two lanes:
     small jobs (n up to 16,384) go whole, all that wait, into one launch
     whenever the small lane is free; large jobs go in arrival order, in
     ranges of a bounded number of pair evaluations per launch (a tick), one
     tick in flight: the next range is issued when the previous one ends, so
     queries issued meanwhile find the device free of job blocks instead of
     behind a queued range.  Large jobs therefore run one after another at
     the device's full rate (the tail of the latency distribution), while
     small jobs and queries run beside them instead of behind them;
  4. completion: finished launches (HIP events) release their memory and
     slots; results are copied out and latencies recorded.
The plain mode is the baseline: one request per launch (``cde_loo_loglik``
or one query launch), in arrival order, each waited for before the next
starts.

Each request's result is computed on the same inputs by the same per-point
arithmetic in either mode, so it is bit-identical alone and in the mix: fused
query launches evaluate each query row independently of the other rows, and
the grouped launch gives each job the totals cde_loo_loglik gives it.
"""
from __future__ import annotations

import collections
import dataclasses
import sys
import time
from typing import Callable

import numpy as np


@dataclasses.dataclass
class ServeRequest:
    rid: int
    kind: str                     # "job" or "query"
    t_arrive: float               # seconds from the start of the run
    footprint: int = 0            # device bytes while in service
    # job payload
    x: np.ndarray | None = None   # [n, dx] float32
    y: np.ndarray | None = None   # [n, 1] float32
    hx: tuple = ()
    hy: tuple = ()
    # query payload
    set_id: int = -1
    xq: np.ndarray | None = None  # [q, dx] float32
    # outcome
    t_admit: float | None = None
    t_done: float | None = None
    result: object = None
    error: str | None = None
    # progress of a job in grouped launches: next point to issue
    next_point: int = 0

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrive


class Executor:
    """Launches work and reports completion; the scheduler owns the policy."""

    def footprint(self, req: ServeRequest) -> int:
        raise NotImplementedError

    def launch_queries(self, set_id: int, reqs: list) -> object:
        """Start one fused launch for `reqs` (same resident set); returns a handle."""
        raise NotImplementedError

    def launch_job(self, req: ServeRequest) -> object:
        """Plain mode: the whole job as one launch."""
        raise NotImplementedError

    def job_points(self, req: ServeRequest) -> int:
        """Number of training points of a job (its n)."""
        return int(req.x.shape[0])

    def round_points(self, req: ServeRequest) -> int:
        """Points per full round of the device for this job's shape: ranges
        of a job are whole multiples of it."""
        return 256

    def prepare_job(self, req: ServeRequest) -> None:
        """Batched mode, at admission: upload the job's data and create its
        model (ordered before its first grouped launch)."""
        raise NotImplementedError

    def launch_job_tick(self, items: list, lane: str = "large") -> object:
        """Batched mode: one grouped launch over work items (req, i0, i1) on
        the given lane ("small": whole small jobs; "large": ranges of large
        jobs, whose successive ranges come in order).  Launches of one lane
        run one after another.  Items that cannot be launched are retried
        alone; those that still fail are returned in the handle's "failed"
        list as (req, message) and are not in flight."""
        raise NotImplementedError

    def done(self, handle) -> bool:
        raise NotImplementedError

    def finish(self, handle) -> None:
        """Copy results of a finished launch into its requests."""
        raise NotImplementedError

    def wait_all(self) -> None:
        pass

    def idle(self) -> None:
        """Called when nothing is in flight (a safe point for deferred frees)."""

    def resident_bytes(self) -> int:
        """Device memory held outside any request (resident sets and their
        scratch); the scheduler admits requests against what remains."""
        return 0


class Scheduler:
    """Admission, batching and completion tracking (device-agnostic)."""

    def __init__(self, executor: Executor, hbm_budget: int, max_active: int = 64,
                 batched: bool = True, clock: Callable[[], float] | None = None,
                 max_query_rows: int = 1 << 16, tick_pairs: float = 3e12,
                 small_job_points: int = 16384, ticks_in_flight: int = 1,
                 grid_cells: int = 256):
        self.ex = executor
        self.max_query_rows = int(max_query_rows)
        # grouped job ticks: pair evaluations per tick (n_range * n * cells),
        # the size up to which a job rides along whole, ticks kept in flight.
        # Ranges are whole rounds of the device (executor.round_points) and
        # about tick_pairs each: every range costs 2-3 ms besides its work
        # (a 200k-point dx = 3 job: 307 ms whole; in ranges of 1, 2, 4 and 7
        # rounds of 16,384 points 341, 326, 317 and 310 ms), while a shorter
        # launch lets queries reach the device sooner.  The default splits a
        # 200k-point 16 x 16 job into three or four ranges.  A second tick in
        # flight keeps the device busy with job blocks back to back; at
        # 50 req/s that raised the query p99 from 0.6 s to 1.4 s.
        self.tick_pairs = float(tick_pairs)
        self.small_job_points = int(small_job_points)
        self.ticks_in_flight = int(ticks_in_flight)
        self.grid_cells = int(grid_cells)
        self.jobs = []          # admitted jobs with ranges still to issue (arrival order)
        self.job_ticks = 0      # grouped launches of large-job ranges in flight
        self.small_busy = False  # a grouped launch of small jobs is in flight
        self.ready_q = collections.OrderedDict()  # set_id -> admitted queries not launched
        self.q_busy = set()                       # sets with a query launch in flight
        self.budget = int(hbm_budget) - int(executor.resident_bytes())
        if self.budget <= 0:
            raise ValueError("the resident sets alone exceed the HBM budget")
        self.max_active = int(max_active)  # slots per request kind (batched mode)
        self.batched = batched
        self.clock = clock or time.perf_counter
        self.pending = collections.deque()   # not yet arrived (sorted by t_arrive)
        # arrived, not admitted: one FIFO queue per request kind
        self.waiting = {"job": collections.deque(), "query": collections.deque()}
        self.inflight = []                   # (handle, [requests])
        self.used = 0
        self.active = 0                      # admitted, not finished (all kinds)
        self.active_kind = {"job": 0, "query": 0}
        self.completed = []
        self.rejected = []
        self.t0 = None
        self._admitted_any = False
        self._seq = 0

    # -------------------------------------------------------------- intake
    def submit_all(self, reqs) -> None:
        for r in sorted(reqs, key=lambda r: r.t_arrive):
            r.footprint = self.ex.footprint(r)
            self.pending.append(r)

    def now(self) -> float:
        return self.clock() - self.t0

    def _arrivals(self, now):
        while self.pending and self.pending[0].t_arrive <= now:
            r = self.pending.popleft()
            if r.footprint > self.budget:
                r.error = "footprint exceeds the HBM budget"
                r.t_done = now
                self.rejected.append(r)
            else:
                self._seq += 1
                self.waiting[r.kind].append((self._seq, r))  # seq: global arrival order

    def n_waiting(self) -> int:
        return sum(len(q) for q in self.waiting.values())

    def _slot_free(self, kind) -> bool:
        if not self.batched:  # plain mode: one request in service at a time
            return self.active == 0
        return self.active_kind[kind] < self.max_active

    def _admit(self, now):
        admitted = []
        while True:
            heads = [q for kind, q in self.waiting.items() if q and self._slot_free(kind)]
            if not heads:
                break
            q = min(heads, key=lambda q: q[0][0])
            if self.used + q[0][1].footprint > self.budget:
                break  # memory in arrival order
            r = q.popleft()[1]
            r.t_admit = now
            self.used += r.footprint
            self.active += 1
            self.active_kind[r.kind] += 1
            admitted.append(r)
        return admitted

    def _job_cells(self, r) -> int:
        cells = len(r.hx) * len(r.hy)
        return cells if cells > 0 else self.grid_cells

    def _is_small(self, r) -> bool:
        return self.ex.job_points(r) <= self.small_job_points

    def _plan_tick(self):
        """Ranges of the oldest large jobs for the next grouped launch, within
        the tick's budget of pair evaluations (range points x n x cells)."""
        items, budget = [], self.tick_pairs
        for r in self.jobs:
            if self._is_small(r):
                continue
            n = self.ex.job_points(r)
            per_point = float(n) * self._job_cells(r)
            rnd = max(256, int(self.ex.round_points(r)) // 256 * 256)
            if items and budget < rnd * per_point:
                break
            take = max(1, int(round(max(budget, 0.0) / (per_point * rnd)))) * rnd
            i1 = min(n, r.next_point + take)
            if n - i1 < rnd // 2:  # no sliver at the end
                i1 = n
            items.append((r, r.next_point, i1))
            budget -= float(i1 - r.next_point) * per_point
        return items

    def _issue(self, items, lane):
        """Launch `items` on `lane`; returns the handle or None, releasing
        the jobs of items that failed."""
        try:
            h = self.ex.launch_job_tick(items, lane)
            failed = {id(r): (r, msg) for r, msg in h.get("failed", [])}
        except Exception as e:  # nothing of the launch is in flight
            h, failed = None, {id(r): (r, str(e)) for r, _, _ in items}
        # a failed item fails only its own job
        self.jobs = [q for q in self.jobs if id(q) not in failed]
        for r, msg in failed.values():
            r.error = f"launch failed: {msg}"
            self._release(r, self.now())
        ok = [(r, i0, i1) for r, i0, i1 in items if id(r) not in failed]
        for r, _, i1 in ok:
            r.next_point = i1
        if h is None:
            return None
        done = [r for r, _, i1 in ok if i1 == self.ex.job_points(r)]
        self.jobs = [r for r in self.jobs if r.next_point < self.ex.job_points(r)]
        self.inflight.append((h, done, "job_" + lane))
        return h

    def _launch_jobs(self):
        if not self.small_busy:
            small = [(r, 0, self.ex.job_points(r)) for r in self.jobs if self._is_small(r)]
            if small and self._issue(small, "small") is not None:
                self.small_busy = True
        while self.job_ticks < self.ticks_in_flight:
            items = self._plan_tick()
            if not items:
                break
            if self._issue(items, "large") is not None:
                self.job_ticks += 1

    def _launch(self, admitted):
        for r in admitted:
            if r.kind == "query":
                self.ready_q.setdefault(r.set_id, []).append(r)
            elif not self.batched:
                self._start(lambda r=r: self.ex.launch_job(r), [r], None)
            else:
                try:
                    self.ex.prepare_job(r)
                    self.jobs.append(r)
                except Exception as e:
                    r.error = f"launch failed: {e}"
                    self._release(r, self.now())
        if self.batched and self.jobs:
            self._launch_jobs()
        for set_id in list(self.ready_q):
            rs = self.ready_q[set_id]
            if not self.batched:
                for r in rs:
                    self._start(lambda s=set_id, r=r: self.ex.launch_queries(s, [r]), [r], None)
                del self.ready_q[set_id]
                continue
            if set_id in self.q_busy or not rs:
                continue
            batch, rows = [], 0
            while rs and (not batch or rows + rs[0].xq.shape[0] <= self.max_query_rows):
                rows += rs[0].xq.shape[0]
                batch.append(rs.pop(0))
            if not rs:
                del self.ready_q[set_id]
            self.q_busy.add(set_id)
            self._start(lambda s=set_id, b=batch: self.ex.launch_queries(s, b), batch, set_id)

    def _start(self, fn, reqs, busy_set):
        try:
            self.inflight.append((fn(), reqs, busy_set))
        except Exception as e:  # a failed launch fails only its own requests
            if busy_set is not None:
                self.q_busy.discard(busy_set)
            for r in reqs:
                r.error = f"launch failed: {e}"
                self._release(r, self.now())

    def _release(self, r, now):
        r.t_done = now
        self.used -= r.footprint
        self.active -= 1
        self.active_kind[r.kind] -= 1
        self.completed.append(r)

    def _complete(self):
        still = []
        for h, reqs, busy_set in self.inflight:
            if self.ex.done(h):
                try:
                    self.ex.finish(h)
                except Exception as e:
                    for r in reqs:
                        r.error = f"completion failed: {e}"
                if busy_set == "job_large":
                    self.job_ticks -= 1
                elif busy_set == "job_small":
                    self.small_busy = False
                elif busy_set is not None:
                    self.q_busy.discard(busy_set)
                now = self.now()
                for r in reqs:
                    self._release(r, now)
            else:
                still.append((h, reqs, busy_set))
        self.inflight = still
        if not still and not self.jobs:
            self.ex.idle()

    def tick(self) -> bool:
        """One scheduling pass; returns False once everything has finished."""
        now = self.now()
        self._admitted_any = False
        self._arrivals(now)
        self._complete()
        if not self.batched and self.inflight:
            return True  # plain mode: one request in service at a time
        admitted = self._admit(now)
        self._admitted_any = bool(admitted)
        if admitted or self.ready_q or self.jobs:
            self._launch(admitted)
        return bool(self.pending or self.n_waiting() or self.inflight or self.ready_q or self.jobs)

    def run(self, idle_sleep: float = 2e-4, deadline: float | None = None,
            progress: float | None = None, log=None) -> None:
        """Drive ticks until every request has finished (or the deadline
        passes).  With ``progress`` (seconds), ``log`` (default: stderr) gets
        a status line at that interval."""
        self.t0 = self.clock()
        next_log = progress
        while self.tick():
            now = self.now()
            if deadline is not None and now > deadline:
                break
            if progress is not None and now >= next_log:
                line = (f"serve: t={now:.0f} s completed={len(self.completed)} "
                        f"waiting={self.n_waiting()} in_flight={sum(len(q) for _, q, _ in self.inflight)}")
                (log or (lambda m: print(m, file=sys.stderr, flush=True)))(line)
                next_log += progress
            if not self._admitted_any:
                time.sleep(idle_sleep)
        self.ex.wait_all()

    # ------------------------------------------------------------- metrics
    def report(self, duration: float) -> dict:
        done = [r for r in self.completed if r.error is None]
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        out = {"completed": len(done), "failed": len(self.completed) - len(done),
               "rejected": len(self.rejected),
               "unfinished": len(self.pending) + self.n_waiting() + len(self.jobs) +
               sum(len(q) for _, q, _ in self.inflight) + sum(len(v) for v in self.ready_q.values())}
        for kind in ("job", "query"):
            lk = np.array([r.latency for r in done if r.kind == kind])
            out[kind] = {"completed": int(lk.size),
                         "p50_s": float(np.percentile(lk, 50)) if lk.size else None,
                         "p99_s": float(np.percentile(lk, 99)) if lk.size else None}
        out["p50_s"] = float(np.percentile(lat, 50)) if lat.size else None
        out["p99_s"] = float(np.percentile(lat, 99)) if lat.size else None
        last = max((r.t_done for r in done), default=0.0)
        out["makespan_s"] = last
        out["throughput_req_s"] = len(done) / max(last, 1e-9)
        out["duration_s"] = duration
        return out


class GpuExecutor(Executor):
    """Runs requests through the C ABI on HIP streams: fused query launches
    on two query streams, grouped job launches (``cde_launch_batch``) on one
    stream per job lane, job uploads on the small-job lane (never behind a
    long launch)."""

    def __init__(self, sets, n_streams: int = 2, grid_points: int = 256, max_query_rows: int = 1 << 16):
        import torch

        from . import _binding
        from .drivers import normal_reference_bandwidths
        from .model import Model, density_summary, launch_batch
        self.torch = torch
        self.Model = Model
        self.B = _binding
        self.density_summary = density_summary
        self.launch_batch = launch_batch
        self.alpha = 0.05
        self.dev = torch.device("cuda:0")
        # Four streams in all: the device runs a process's work on four
        # hardware queues, and streams that share a queue run in order, so a
        # fifth stream would put a long job launch in front of a short query
        # launch.  Two query streams, the small-job lane (which also carries
        # job uploads: short work) and the large-job lane.
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_streams)]
        self.job_streams = {"small": torch.cuda.Stream(device=self.dev),
                            "large": torch.cuda.Stream(device=self.dev)}
        self.upload_stream = self.job_streams["small"]
        self.rr = 0
        self._round = {}     # (dx, dy) -> points per full round of the grouped grid pass
        self.job_state = {}  # rid -> {"model", "totals", "keep", "ready" event}
        # Finished job models are destroyed only when the device is idle (or
        # in bulk past a limit): freeing device memory synchronises the whole
        # device and would serialise the overlapping launches.
        self.graveyard = []
        self.graveyard_limit = 64
        self.sets = []
        for x, y in sets:
            x32 = np.ascontiguousarray(x, dtype=np.float32)
            y32 = np.ascontiguousarray(y, dtype=np.float32).reshape(len(x32), -1)
            m = Model(torch.from_numpy(x32).to(self.dev), torch.from_numpy(y32).to(self.dev))
            h = normal_reference_bandwidths(x32.astype(np.float64), y32.astype(np.float64)).tolist()
            ys = y32[:, 0].astype(np.float64)
            yg = np.linspace(ys.min() - 3 * ys.std(), ys.max() + 3 * ys.std(), grid_points)
            ygd = torch.from_numpy(yg.astype(np.float32).reshape(-1, 1)).to(self.dev)
            yg64 = torch.from_numpy(yg.astype(np.float32).astype(np.float64)).to(self.dev)
            self.sets.append({"model": m, "h": h, "ygrid": ygd, "ygrid64": yg64, "k": grid_points,
                              "dx": x32.shape[1]})
            # One fused batch of the largest size the scheduler forms grows
            # the set's scratch to its final size now: later queries then
            # never reallocate (a device-wide synchronisation), and the
            # memory is counted in resident_bytes.
            xw = torch.from_numpy(np.repeat(x32[:1], max_query_rows, axis=0)).to(self.dev)
            f = m.query(xw, ygd, h)
            m.conditional_mean(xw, h)
            density_summary(f, yg64, self.alpha)
            del xw, f
        torch.cuda.synchronize()
        self._resident = sum(st["model"].device_bytes for st in self.sets)

    def _stream(self):
        s = self.streams[self.rr % len(self.streams)]
        self.rr += 1
        return s

    def resident_bytes(self) -> int:
        return self._resident

    def footprint(self, r):
        if r.kind == "query":
            k = self.sets[r.set_id]["k"]
            return int(r.xq.shape[0]) * (k * 8 + 128) + 4096
        n, dx = r.x.shape
        dy = r.y.shape[1] if r.y.ndim > 1 else 1
        return self.B.workspace_bytes(n, dx, dy, self.B.CDE_F32, len(r.hx), len(r.hy)) + (1 << 20)

    def launch_queries(self, set_id, reqs):
        torch = self.torch
        st = self.sets[set_id]
        s = self._stream()
        with torch.cuda.stream(s):
            xq = np.concatenate([r.xq for r in reqs]).astype(np.float32)
            xqd = torch.from_numpy(xq).to(self.dev, non_blocking=False)
            f = st["model"].query(xqd, st["ygrid"], st["h"], stream=s)
            # query-side products: E[y|x], mass, mode and the narrowest
            # (1 - alpha) interval of each row (per-row results, so fusing
            # requests changes no bit)
            mean = st["model"].conditional_mean(xqd, st["h"], stream=s)
            summ = self.density_summary(f, st["ygrid64"], self.alpha, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"ev": ev, "f": f, "mean": mean, "summary": summ, "reqs": reqs, "keep": xqd}

    def launch_job(self, r):
        torch = self.torch
        s = self._stream()
        with torch.cuda.stream(s):
            xd = torch.from_numpy(r.x).to(self.dev)
            yd = torch.from_numpy(r.y).to(self.dev)
            m = self.Model(xd, yd, stream=s)
            tot, _, _ = m.loo_grid(r.hx, r.hy, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"ev": ev, "tot": tot, "model": m, "req": r, "keep": (xd, yd)}

    def round_points(self, r):
        key = (r.x.shape[1], r.y.shape[1] if r.y.ndim > 1 else 1)
        if key not in self._round:
            self._round[key] = int(self.B.load().cde_batch_round_points(*key)) or 256
        return self._round[key]

    def prepare_job(self, r):
        torch = self.torch
        u = self.upload_stream
        with torch.cuda.stream(u):
            xd = torch.from_numpy(r.x).to(self.dev)
            yd = torch.from_numpy(r.y).to(self.dev)
            m = self.Model(xd, yd, stream=u)
            totals = torch.empty(len(r.hx) * len(r.hy), dtype=torch.float64, device=self.dev)
            ready = torch.cuda.Event()
            ready.record(u)
        self.job_state[r.rid] = {"model": m, "totals": totals, "keep": (xd, yd), "ready": ready}

    def launch_job_tick(self, items, lane="large"):
        torch = self.torch
        s = self.job_streams[lane]
        for r, i0, _ in items:
            if i0 == 0:  # the job's upload and model creation come first
                s.wait_event(self.job_state[r.rid]["ready"])
        groups = {}
        for r, i0, i1 in items:
            key = (r.x.shape[1], r.y.shape[1] if r.y.ndim > 1 else 1, tuple(r.hx), tuple(r.hy))
            groups.setdefault(key, []).append((r, i0, i1))
        failed = []

        def work(r, i0, i1):
            js = self.job_state[r.rid]
            return (js["model"], i0, i1, js["totals"] if i1 == r.x.shape[0] else None, None)

        with torch.cuda.stream(s):
            for (_, _, hx, hy), its in groups.items():
                try:
                    self.launch_batch([work(*it) for it in its], hx, hy, stream=s)
                except Exception:
                    # the library checks every item before it launches any,
                    # so nothing of this group ran: each item alone
                    for it in its:
                        try:
                            self.launch_batch([work(*it)], hx, hy, stream=s)
                        except Exception as e:
                            failed.append((it[0], str(e)))
            ev = torch.cuda.Event()
            ev.record(s)
        bad = {id(r) for r, _ in failed}
        for r, _ in failed:
            self.graveyard.append(self.job_state.pop(r.rid)["model"])
        tick = [(r, i1 == r.x.shape[0]) for r, _, i1 in items if id(r) not in bad]
        return {"ev": ev, "tick": tick, "failed": failed}

    def done(self, h):
        return h["ev"].query()

    def finish(self, h):
        if "f" in h:
            f = h["f"].cpu().numpy()
            mean = h["mean"].cpu().numpy()
            summ = h["summary"].cpu().numpy()
            o = 0
            for r in h["reqs"]:
                q = r.xq.shape[0]
                r.result = {"f": f[o:o + q], "mean": mean[o:o + q], "summary": summ[o:o + q]}
                o += q
        elif "tick" in h:
            for r, last in h["tick"]:
                if not last:
                    continue
                js = self.job_state.pop(r.rid)
                self._job_result(r, js["totals"].cpu().numpy())
                self.graveyard.append(js["model"])
            if len(self.graveyard) >= self.graveyard_limit:
                self.idle()
        else:
            r = h["req"]
            self._job_result(r, h["tot"].cpu().numpy())
            self.graveyard.append(h["model"])
            if len(self.graveyard) >= self.graveyard_limit:
                self.idle()

    @staticmethod
    def _job_result(r, t):
        finite = np.where(np.isfinite(t), t, -np.inf)
        r.result = {"totals": t.reshape(len(r.hx), len(r.hy)), "argmax": int(np.argmax(finite))}

    def idle(self):
        for m in self.graveyard:
            m.close()
        self.graveyard = []

    def wait_all(self):
        self.torch.cuda.synchronize()
        self.idle()
