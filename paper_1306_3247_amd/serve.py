"""Continuous-batching server of split-operator solves on one GPU.

Requests (a grid, a potential, a Gaussian initial state and a step count)
arrive over time.  A request is admitted when its device bytes (state plus
tables, `wp_workspace_bytes`, the memory estimate of Section 3.5) fit in the
HBM budget next to the solves already resident; its state then stays on the
device until it has taken all its steps.  Every tick advances the resident
solves together: those with at least `tick_steps` steps left run in one
batch (`wp_batch_propagate`, shared launches), those with fewer left take
their remaining steps in their own launches and retire.  A retired state is
copied to pinned host memory on a second stream, overlapped with the next
ticks; its latency ends when that copy has landed.

All arithmetic runs in the HIP kernels of libwavepacket; this module only
schedules.  Membership changes create a new batch; a batch or a solve that
is no longer used is kept until the device has drained (freeing device
memory synchronises the device), which happens when the server is idle, when
memory is needed for the next admission, or after `flush_objects` of them.
"""
from __future__ import annotations

import dataclasses as dc
import time
from collections import deque
from typing import Deque, List, Optional

import numpy as np

from . import sim as _sim


@dc.dataclass
class Served:
    """One served request: times in seconds from the start of the run."""
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    steps: int = 0
    sites: int = 0
    bytes: int = 0
    chunks: List[int] = dc.field(default_factory=list)  # step counts of its propagate calls
    result: Optional[np.ndarray] = None  # final state (complex64/128), if kept
    rejected: bool = False

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dc.dataclass
class Report:
    served: List[Served]
    makespan: float
    ticks: int
    batches: int
    flushes: int
    peak_bytes: int
    budget: int

    def latencies(self, first_rid: int = 0) -> np.ndarray:
        return np.array([s.latency for s in self.served if not s.rejected and s.rid >= first_rid])

    def summary(self, first_rid: int = 0) -> dict:
        """Statistics over the requests with rid >= first_rid (earlier ones
        warm the server up); throughput over the span from their first
        arrival to their last result."""
        lat = self.latencies(first_rid)
        done = [s for s in self.served if not s.rejected and s.rid >= first_rid]
        site_steps = float(sum(s.sites * s.steps for s in done))
        span = (max(s.finished for s in done) - min(s.arrival for s in done)) if done else 0.0
        return {
            "requests": len(done),
            "rejected": sum(1 for s in self.served if s.rejected and s.rid >= first_rid),
            "makespan_s": span,
            "requests_per_s": len(done) / span if span > 0 else 0.0,
            "site_steps_per_s": site_steps / span if span > 0 else 0.0,
            "p50_s": float(np.percentile(lat, 50)) if lat.size else float("nan"),
            "p99_s": float(np.percentile(lat, 99)) if lat.size else float("nan"),
            "mean_queue_s": float(np.mean([s.admitted - s.arrival for s in done])) if done else float("nan"),
            "ticks": self.ticks,
            "batches": self.batches,
            "flushes": self.flushes,
            "peak_bytes": self.peak_bytes,
            "budget_bytes": self.budget,
        }


class _Job:
    __slots__ = ("rec", "prob", "sim", "left", "host", "copy_event")

    def __init__(self, rec: Served, prob):
        self.rec, self.prob = rec, prob
        self.sim = None
        self.left = 0
        self.host = None
        self.copy_event = None


class Server:
    """Admission by HBM budget, continuous batching, asynchronous retirement.

    budget_bytes  device bytes the resident solves may hold together
    tick_steps    steps per batched tick (members with fewer left finish alone)
    graph_steps   steady steps per captured graph inside a batch (0: direct launches)
    max_active    resident solves at most
    depth         ticks enqueued ahead of the one the host waits for
    keep_results  keep final states on the host: True for all, or a set of rids
    """

    def __init__(self, budget_bytes: int = 192 << 30, tick_steps: int = 256, graph_steps: int = 16,
                 max_active: int = 256, depth: int = 2, flush_objects: int = 32, keep_results: bool = False):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        if tick_steps < 1 or depth < 1 or max_active < 1:
            raise ValueError("tick_steps, depth and max_active must be >= 1")
        self.torch = torch
        self.budget = int(budget_bytes)
        self.tick_steps = int(tick_steps)
        self.graph_steps = int(graph_steps)
        self.max_active = int(max_active)
        self.depth = int(depth)
        self.flush_objects = int(flush_objects)
        self.keep_results = keep_results
        self.stream = torch.cuda.Stream()       # all solver work
        self.copy_stream = torch.cuda.Stream()  # device-to-host copies of results

    # -- helpers ---------------------------------------------------------
    @staticmethod
    def request_bytes(prob) -> int:
        return _sim.workspace_bytes(prob.grid, prob.precision)

    def _admit(self, job: _Job, now: float) -> None:
        torch = self.torch
        p = job.prob
        with torch.cuda.stream(self.stream):
            s = _sim.Simulation(p.grid, p.pot, p.precision, stream=self.stream)
            s.set_gaussian(p.init.center, p.init.sigma, p.init.k, p.t0)
        job.sim = s
        job.left = int(p.steps)
        job.rec.admitted = now

    def _start_copy(self, job: _Job, after) -> None:
        torch = self.torch
        buf = job.sim.buffer
        job.host = torch.empty(buf.numel(), dtype=torch.uint8, pin_memory=True)
        self.copy_stream.wait_event(after)
        with torch.cuda.stream(self.copy_stream):
            job.host.copy_(buf, non_blocking=True)
            buf.record_stream(self.copy_stream)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        job.copy_event = ev

    def _finish(self, job: _Job, now: float) -> None:
        rec = job.rec
        rec.finished = now
        keep = self.keep_results
        if keep is True or (keep and rec.rid in keep):
            dt = np.complex128 if job.prob.precision == "c128" else np.complex64
            shape = job.sim.shape
            pitch = _sim.state_pitch(job.prob.grid, job.prob.precision)
            plane = int(np.prod(shape[1:]))
            flat = job.host.numpy().view(dt)[: shape[0] * pitch]
            rec.result = flat.reshape(shape[0], pitch)[:, :plane].reshape(shape).copy()
        job.host = None

    # -- the loop ----------------------------------------------------------
    def run(self, requests, progress=None) -> Report:
        """Serve `requests` (objects with .rid, .arrival in seconds, .problem),
        replaying their arrival times against the wall clock.  progress, if
        given, is called as progress(finished, total, seconds) whenever a
        result has reached the host."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        served = [Served(r.rid, float(r.arrival), steps=int(r.problem.steps),
                         sites=int(r.problem.grid.points()), bytes=self.request_bytes(r.problem)) for r in reqs]
        pending: Deque[_Job] = deque()
        active: List[_Job] = []
        retiring: List[_Job] = []
        grave_sims: List[_Job] = []
        grave_batches: list = []
        inflight: Deque = deque()
        batch, batch_key = None, None
        used = peak = 0
        ticks = batches = flushes = 0
        finished = 0
        nxt = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0

        def flush() -> None:
            nonlocal used, flushes
            if not grave_sims and not grave_batches:
                return
            self.stream.synchronize()
            for b in grave_batches:
                b.close()
            grave_batches.clear()
            for j in grave_sims:
                j.sim.close()
                j.sim = None
                used -= j.rec.bytes
            grave_sims.clear()
            flushes += 1

        while nxt < len(reqs) or pending or active or retiring:
            now = clock()
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                job = _Job(served[nxt], reqs[nxt].problem)
                if job.rec.bytes > self.budget:
                    job.rec.rejected = True
                else:
                    pending.append(job)
                nxt += 1
            # results that have reached the host
            still = []
            for j in retiring:
                if j.copy_event.query():
                    self._finish(j, clock())
                    grave_sims.append(j)
                    finished += 1
                    if progress is not None:
                        progress(finished, len(reqs), clock())
                else:
                    still.append(j)
            retiring = still
            # admission, first come first served
            while pending and len(active) < self.max_active:
                need = pending[0].rec.bytes
                if used + need > self.budget:
                    if grave_sims:
                        flush()
                        continue
                    break
                job = pending.popleft()
                self._admit(job, clock())
                used += need
                peak = max(peak, used)
                active.append(job)
            if len(grave_sims) + len(grave_batches) >= self.flush_objects:
                flush()

            if active:
                long_ = [j for j in active if j.left >= self.tick_steps]
                tail = [j for j in active if j.left < self.tick_steps]
                key = tuple(id(j) for j in long_)
                if long_ and key != batch_key:
                    if batch is not None:
                        grave_batches.append(batch)
                    batch = _sim.Batch([j.sim for j in long_], stream=self.stream, graph_steps=self.graph_steps)
                    batch_key = key
                    batches += 1
                if long_:
                    batch.propagate(self.tick_steps)
                    for j in long_:
                        j.left -= self.tick_steps
                        j.rec.chunks.append(self.tick_steps)
                for j in tail:
                    j.sim.propagate(j.left)
                    j.rec.chunks.append(j.left)
                    j.left = 0
                ev = torch.cuda.Event()
                ev.record(self.stream)
                inflight.append(ev)
                ticks += 1
                done = [j for j in active if j.left == 0]
                for j in done:
                    self._start_copy(j, ev)
                retiring.extend(done)
                active = [j for j in active if j.left > 0]
                if not long_ and batch is not None:
                    grave_batches.append(batch)
                    batch, batch_key = None, None
                while len(inflight) > self.depth:
                    inflight.popleft().synchronize()
            else:
                # Nothing to advance: drain, free what is unused, then wait
                # for a copy or the next arrival.
                while inflight:
                    inflight.popleft().synchronize()
                if batch is not None:
                    grave_batches.append(batch)
                    batch, batch_key = None, None
                flush()
                if retiring:
                    retiring[0].copy_event.synchronize()
                elif not pending and nxt < len(reqs):
                    wait = reqs[nxt].arrival - clock()
                    if wait > 0:
                        time.sleep(wait)
                elif pending:
                    # The head does not fit although nothing else is resident.
                    j = pending.popleft()
                    j.rec.rejected = True
        while inflight:
            inflight.popleft().synchronize()
        if batch is not None:
            grave_batches.append(batch)
        flush()
        makespan = clock()
        return Report(served, makespan, ticks, batches, flushes, peak, self.budget)


def capacity(requests, **server_args) -> float:
    """Closed-loop capacity in requests per second: every request present at
    time zero."""
    closed = [dc.replace(r, arrival=0.0) for r in requests]
    rep = Server(**server_args).run(closed)
    return rep.summary()["requests_per_s"]


def sweep(make_requests, rates, **server_args) -> list:
    """Serve one request stream per arrival rate; make_requests(rate, i)
    returns the stream for the i-th rate.  Returns one summary per rate."""
    out = []
    for i, r in enumerate(rates):
        rep = Server(**server_args).run(make_requests(r, i))
        s = rep.summary()
        s["rate_hz"] = r
        out.append(s)
    return out
