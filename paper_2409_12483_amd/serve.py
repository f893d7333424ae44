"""Continuous-batching service for ADER-DG solve requests.

Requests (PDE, degree N, cells, number of steps) arrive over time.  The
scheduler admits them first-come first-served while two budgets hold: device
memory (each request holds its state and the library's ping-pong copy) and a
slot limit on concurrently active requests.  Requests admitted together with
the same (PDE, N) form a cohort, i.e. one library handle and one kernel
launch per step for all of them.

There is no global tick.  Every cohort runs on one of a few device streams
and advances in chunks: a chunk is the smallest number of steps any of its
unfinished requests still needs (capped), enqueued with an event behind it.
The loop polls the events without blocking; when a cohort's chunk is done it
retires the requests that have run all their steps (their end time is
frozen, so they stop advancing), frees the cohort once all its requests are
done (stream-ordered: no host synchronisation), and enqueues the next chunk.
New arrivals are admitted as soon as slots and memory free up, and their
cohorts start at once on the streams, overlapping the cohorts already
running.  A request's numbers never depend on the other requests of its
cohort or on the other cohorts: each problem of a launch reads only its own
state and clock.

The scheduler talks to an executor (``GpuExecutor`` here; tests use a CPU
stand-in with the same methods):
    create(specs) -> cohort      step(cohort, n)      ready(cohort)
    freeze(cohort, idx)          status(cohort)       state(cohort, i)
    free(cohort)                 wait(timeout)
"""

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import batch as B


@dataclass
class Request:
    id: int
    arrival: float
    pde: str
    N: int
    ncells: int
    steps: int
    k: int = 1
    phase: float = 0.0
    admitted: float = None
    done: float = None
    steps_done: int = 0

    @property
    def spec(self):
        return {"pde": self.pde, "N": self.N, "ncells": self.ncells, "k": self.k,
                "phase": self.phase}

    @property
    def nbytes(self):
        return B.state_bytes(self.spec)

    @property
    def dofs(self):
        return self.ncells * (self.N + 1) * 3


@dataclass
class Cohort:
    requests: list
    handle: object
    remaining: list = field(default_factory=list)   # steps not yet enqueued, per request
    chunks: deque = field(default_factory=deque)    # (event, steps, advanced, finishing) in flight

    def active(self):
        return [i for i, r in enumerate(self.remaining) if r > 0]


def cfl_for(N):
    """Courant number of a request: 0.4, or 0.3 for N >= 8, where 0.4 lies
    beyond the scheme's stability bound."""
    return 0.4 if N <= 7 else 0.3


class GpuExecutor:
    """Cohorts as library handles spread over a few device streams (default
    priority; a new cohort takes the stream with the fewest live cohorts)."""

    def __init__(self, precision=None, streams=4, poll_s=2e-4):
        import torch
        from . import abi
        self.torch = torch
        self.precision = abi.FP64 if precision is None else precision
        self.streams = [torch.cuda.Stream() for _ in range(max(1, int(streams)))]
        self.load = [0] * len(self.streams)
        self.poll_s = poll_s

    def create(self, specs):
        cfls = {cfl_for(s["N"]) for s in specs}
        assert len(cfls) == 1, "a cohort shares one degree"
        k = min(range(len(self.streams)), key=lambda i: self.load[i])
        self.load[k] += 1
        b = B.Batch(specs, precision=self.precision, stream=self.streams[k], cfl=cfls.pop())
        b.slot = k
        return b

    def step(self, cohort, n):
        """Enqueue n steps; returns the event that marks their end."""
        cohort.step(n)
        return cohort.event

    def ready(self, event):
        return event.query()

    def wait(self, timeout):
        time.sleep(max(0.0, min(timeout, self.poll_s)))

    def freeze(self, cohort, idx):
        cohort.freeze(idx)

    def status(self, cohort):
        """Most severe status of each problem over every call so far (read
        after the cohort's last event completed)."""
        return cohort.sticky.cpu().numpy()

    def state(self, cohort, i):
        return cohort.u[i].cpu().numpy()

    def free(self, cohort):
        self.load[cohort.slot] -= 1
        cohort.close()


class Scheduler:
    def __init__(self, executor, hbm_budget=200e9, max_active=256, max_steps_per_tick=500,
                 clock=time.perf_counter, keep_states=False, admit_window=2e-3, idle_cohorts=2,
                 chunk_dof_steps=1e8, depth=2):
        self.ex = executor
        self.depth = max(1, int(depth))      # chunks in flight per cohort
        # a chunk holds about chunk_dof_steps DoF-updates (a few milliseconds
        # of device time), so that no cohort holds its stream for long
        self.chunk_work = float(chunk_dof_steps)
        # arrivals wait at most admit_window seconds to be admitted together
        # (one cohort, one launch per step), and are admitted at once while
        # fewer than idle_cohorts cohorts are running
        self.window = float(admit_window)
        self.idle = int(idle_cohorts)
        self.budget = float(hbm_budget)
        self.max_active = int(max_active)
        self.cap = int(max_steps_per_tick)
        self.clock = clock
        self.keep = keep_states
        self.queue = []          # waiting requests, FIFO
        self.cohorts = []
        self.used = 0.0
        self.nactive = 0
        self.finished = []
        self.states = {}
        self.bad = {}
        self.ticks = 0           # chunks enqueued
        self.max_inflight = 0    # most cohorts with work on the device at once

    # -- admission -------------------------------------------------------
    def head_fits(self):
        r = self.queue[0]
        return self.nactive + 1 <= self.max_active and self.used + r.nbytes <= self.budget

    def submit(self, req):
        if req.nbytes > self.budget:
            raise ValueError(f"request {req.id} needs {req.nbytes} bytes, over the whole budget")
        self.queue.append(req)

    def admit(self, now):
        took = []
        while self.queue:
            r = self.queue[0]
            if self.nactive + 1 > self.max_active or self.used + r.nbytes > self.budget:
                break            # first come, first served: the head waits for room
            self.queue.pop(0)
            r.admitted = now
            self.used += r.nbytes
            self.nactive += 1
            took.append(r)
        groups = {}
        for r in took:
            groups.setdefault((r.pde, r.N), []).append(r)
        for reqs in groups.values():
            h = self.ex.create([r.spec for r in reqs])
            self.cohorts.append(Cohort(reqs, h, [r.steps for r in reqs]))
        return took

    # -- chunks: enqueue, and retire when done -----------------------------
    def launch(self):
        """Keep `depth` chunks in flight per cohort.  The requests a chunk
        finishes are frozen right behind it in stream order, so the next chunk
        can be enqueued before the host has seen the first one end."""
        for c in self.cohorts:
            while len(c.chunks) < self.depth:
                act = c.active()
                if not act:
                    break
                work = sum(c.requests[i].dofs for i in act)
                n = min(min(c.remaining[i] for i in act), self.cap, max(1, int(self.chunk_work // work)))
                ev = self.ex.step(c.handle, n)
                fin = []
                for i in act:
                    c.remaining[i] -= n
                    if c.remaining[i] == 0:
                        fin.append(i)
                if fin and len(fin) < len(act):
                    self.ex.freeze(c.handle, fin)
                c.chunks.append((ev, n, act, fin))
                self.ticks += 1
        self.max_inflight = max(self.max_inflight, sum(1 for c in self.cohorts if c.chunks))

    def complete(self):
        """Retire the requests of the chunks that have finished, free the
        cohorts that are done.  Returns the number of chunks retired."""
        retired = 0
        keep = []
        for c in self.cohorts:
            while c.chunks and self.ex.ready(c.chunks[0][0]):
                _, n, act, fin = c.chunks.popleft()
                retired += 1
                now = self.clock()
                for i in act:
                    c.requests[i].steps_done += n
                if fin:
                    st = self.ex.status(c.handle)
                    for i in fin:
                        r = c.requests[i]
                        r.done = now
                        self.finished.append(r)
                        if st[i] != 0:
                            self.bad[r.id] = int(st[i])
                        if self.keep:
                            self.states[r.id] = self.ex.state(c.handle, i)
            if c.chunks or c.active():
                keep.append(c)
            else:
                self.ex.free(c.handle)
                for r in c.requests:
                    self.used -= r.nbytes
                    self.nactive -= 1
        self.cohorts = keep
        return retired

    # -- the service loop over an arrival trace --------------------------
    def run(self, requests):
        """Serve requests (arrival times in seconds from the start); returns metrics."""
        pending = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        base = self.clock
        self.clock = lambda: base() - t0
        try:
            j = 0
            while j < len(pending) or self.queue or self.cohorts:
                now = self.clock()
                while j < len(pending) and pending[j].arrival <= now:
                    self.submit(pending[j])
                    j += 1
                if self.queue and (len(self.cohorts) < self.idle
                                   or now >= self.queue[0].arrival + self.window):
                    self.admit(now)
                self.launch()
                if not self.complete():
                    # sleep until the next arrival, the queue head's admission
                    # deadline (if it fits), or a chunk finishing
                    wake = [pending[j].arrival] if j < len(pending) else []
                    if self.queue and self.head_fits():
                        wake.append(self.queue[0].arrival + self.window)
                    t = min(wake) - self.clock() if wake else 1.0
                    self.ex.wait(min(max(0.0, t), 1.0))
            makespan = self.clock()
        finally:
            self.clock = base
        out = summarize(self.finished, makespan, self.ticks)
        out["max_cohorts_in_flight"] = self.max_inflight
        return out


def summarize(finished, makespan, ticks):
    lat = np.array([r.done - r.arrival for r in finished])
    que = np.array([r.admitted - r.arrival for r in finished])
    svc = np.array([r.done - r.admitted for r in finished])
    dof = float(sum(r.dofs * r.steps for r in finished))
    pct = lambda a, q: round(float(np.percentile(a, q)) * 1e3, 2) if len(a) else None
    return {"requests": len(finished), "makespan_s": round(makespan, 3), "ticks": ticks,
            "dof_updates_per_s": round(dof / makespan, 1) if makespan > 0 else None,
            "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
            "queue_ms": {"p50": pct(que, 50), "p99": pct(que, 99)},
            "service_ms": {"p50": pct(svc, 50), "p99": pct(svc, 99)}}


def requests_from_trace(trace):
    return [Request(id=t["id"], arrival=t["arrival"], pde=t["pde"], N=t["N"], ncells=t["ncells"],
                    steps=t["steps"], k=t.get("k", 1), phase=t.get("phase", 0.0)) for t in trace]
