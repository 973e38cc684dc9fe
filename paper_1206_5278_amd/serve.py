"""Continuous-batching server for bandwidth-selection jobs and conditional
density queries (the estimator of eq. 1 and the criterion of eq. 3).

Two request kinds:
  * job   -- exact LOO log-likelihood over a scalar bandwidth grid on the
             request's own training set (``cde_create`` + ``cde_loo_loglik``);
             the answer is the grid of totals and its argmax.
  * query -- f(y | x) for q query points on a y-grid against one of the
             resident training sets (``cde_density_query``).

Scheduling (one scheduler thread, ``tick`` is one pass):
  1. arrivals whose time has come enter the waiting queue (FIFO);
  2. admission: requests leave the queue in order while their device-memory
     footprint fits the HBM budget and a slot is free -- requests arriving
     while others run are admitted as slots and memory free up;
  3. launch: admitted queries wait in a per-set ready list; whenever a
     resident set has no query launch in flight, all of its ready queries
     become ONE fused query launch (so queries that arrive while a batch runs
     join the next batch); each admitted job is launched on the next of
     several streams, so jobs of different sizes overlap on the device with
     each other and with the queries;
  4. completion: finished launches (HIP events) release their memory and
     slots; results are copied out and latencies recorded.
The plain mode is the baseline: one request per launch, in arrival order,
each waited for before the next starts.

Each request's result is computed by the same kernels on the same inputs in
either mode, so it is identical alone and in the mix (fused query launches
evaluate each query row independently of the other rows).
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
                 max_query_rows: int = 1 << 16):
        self.ex = executor
        self.max_query_rows = int(max_query_rows)
        self.ready_q = collections.OrderedDict()  # set_id -> admitted queries not launched
        self.q_busy = set()                       # sets with a query launch in flight
        self.budget = int(hbm_budget) - int(executor.resident_bytes())
        if self.budget <= 0:
            raise ValueError("the resident sets alone exceed the HBM budget")
        self.max_active = int(max_active)
        self.batched = batched
        self.clock = clock or time.perf_counter
        self.pending = collections.deque()   # not yet arrived (sorted by t_arrive)
        self.waiting = collections.deque()   # arrived, not admitted
        self.inflight = []                   # (handle, [requests])
        self.used = 0
        self.active = 0
        self.completed = []
        self.rejected = []
        self.t0 = None

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
                self.waiting.append(r)

    def _admit(self, now):
        admitted = []
        limit = self.max_active if self.batched else 1
        while self.waiting and self.active < limit and \
                self.used + self.waiting[0].footprint <= self.budget:
            r = self.waiting.popleft()
            r.t_admit = now
            self.used += r.footprint
            self.active += 1
            admitted.append(r)
        return admitted

    def _launch(self, admitted):
        for r in admitted:
            if r.kind == "query":
                self.ready_q.setdefault(r.set_id, []).append(r)
            else:
                self._start(lambda r=r: self.ex.launch_job(r), [r], None)
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
                if busy_set is not None:
                    self.q_busy.discard(busy_set)
                now = self.now()
                for r in reqs:
                    self._release(r, now)
            else:
                still.append((h, reqs, busy_set))
        self.inflight = still
        if not still:
            self.ex.idle()

    def tick(self) -> bool:
        """One scheduling pass; returns False once everything has finished."""
        now = self.now()
        self._arrivals(now)
        self._complete()
        if not self.batched and self.inflight:
            return True  # plain mode: one request in service at a time
        admitted = self._admit(now)
        if admitted or self.ready_q:
            self._launch(admitted)
        return bool(self.pending or self.waiting or self.inflight or self.ready_q)

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
                        f"waiting={len(self.waiting)} in_flight={sum(len(q) for _, q, _ in self.inflight)}")
                (log or (lambda m: print(m, file=sys.stderr, flush=True)))(line)
                next_log += progress
            if not self.waiting or self.active >= self.max_active:
                time.sleep(idle_sleep)
        self.ex.wait_all()

    # ------------------------------------------------------------- metrics
    def report(self, duration: float) -> dict:
        done = [r for r in self.completed if r.error is None]
        lat = np.array([r.latency for r in done]) if done else np.zeros(0)
        out = {"completed": len(done), "failed": len(self.completed) - len(done),
               "rejected": len(self.rejected),
               "unfinished": len(self.pending) + len(self.waiting) +
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
    """Runs requests through the C ABI on HIP streams."""

    def __init__(self, sets, n_streams: int = 4, grid_points: int = 256, max_query_rows: int = 1 << 16):
        import torch

        from . import _binding
        from .drivers import normal_reference_bandwidths
        from .model import Model, density_summary
        self.torch = torch
        self.Model = Model
        self.B = _binding
        self.density_summary = density_summary
        self.alpha = 0.05
        self.dev = torch.device("cuda:0")
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_streams)]
        self.rr = 0
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
        else:
            r = h["req"]
            t = h["tot"].cpu().numpy()
            finite = np.where(np.isfinite(t), t, -np.inf)
            r.result = {"totals": t.reshape(len(r.hx), len(r.hy)), "argmax": int(np.argmax(finite))}
            self.graveyard.append(h["model"])
            if len(self.graveyard) >= self.graveyard_limit:
                self.idle()

    def idle(self):
        for m in self.graveyard:
            m.close()
        self.graveyard = []

    def wait_all(self):
        self.torch.cuda.synchronize()
        self.idle()

