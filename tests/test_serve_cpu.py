"""Scheduler logic of the serving loop, with a CPU stand-in executor and a
virtual clock (no GPU): admission budgets, first-come-first-served order,
cohort grouping, exact step counts per request, latency bookkeeping."""

import numpy as np
import pytest

from paper_2409_12483_amd import serve
from paper_2409_12483_amd import workloads as W


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeExecutor:
    """Counts the steps each problem is advanced by; a chunk occupies one of
    `streams` simulated device streams for work / rate seconds of the
    virtual clock, and chunks on different streams overlap."""

    def __init__(self, clock, dof_rate=1e9, streams=4, fail=None):
        self.clock = clock
        self.rate = dof_rate
        self.busy = [0.0] * streams
        self.load = [0] * streams
        self.live = []
        self.max_live_problems = 0
        self.max_live_bytes = 0
        self.created = []
        self.fail = dict(fail or {})      # (cohort index, problem, chunk) -> status planted there

    def create(self, specs):
        k = min(range(len(self.busy)), key=lambda i: self.load[i])
        self.load[k] += 1
        c = {"specs": list(specs), "steps": [0] * len(specs), "frozen": [False] * len(specs),
             "freed": False, "slot": k, "done_at": 0.0, "chunks": 0,
             "sticky": np.zeros(len(specs), dtype=np.int32), "index": len(self.created)}
        self.live.append(c)
        self.created.append(c)
        self.max_live_problems = max(self.max_live_problems, sum(len(x["specs"]) for x in self.live))
        self.max_live_bytes = max(self.max_live_bytes, sum(serve.B.state_bytes(s) for x in self.live
                                                            for s in x["specs"]))
        return c

    def step(self, c, n):
        assert n >= 1 and not c["freed"]
        work = 0.0
        for i, s in enumerate(c["specs"]):
            if not c["frozen"][i]:
                c["steps"][i] += n
                work += s["ncells"] * (s["N"] + 1) * 3 * n
                st = self.fail.get((c["index"], i, c["chunks"]), 0)
                c["sticky"][i] = min(c["sticky"][i], st)
        k = c["slot"]
        start = max(self.clock.t, self.busy[k])
        self.busy[k] = start + work / self.rate
        c["done_at"] = self.busy[k]
        c["chunks"] += 1
        return c["done_at"]

    def ready(self, done_at):
        return self.clock.t >= done_at

    def wait(self, timeout):
        later = [c["done_at"] for c in self.live if c["done_at"] > self.clock.t]
        step = min([timeout] + [t - self.clock.t for t in later])
        self.clock.t += max(step, 0.0)

    def freeze(self, c, idx):
        for i in idx:
            c["frozen"][i] = True

    def status(self, c):
        return c["sticky"].copy()

    def state(self, c, i):
        return np.array([c["steps"][i]])

    def free(self, c):
        c["freed"] = True
        self.load[c["slot"]] -= 1
        self.live.remove(c)


def _trace(n=60, rate=50.0, seed=1):
    return serve.requests_from_trace(W.request_trace(nreq=n, rate=rate, seed=seed, cmin=1000,
                                                     cmax=20000, smin=5, smax=60))


def _run(reqs, fail=None, streams=4, **kw):
    clk = VirtualClock()
    ex = FakeExecutor(clk, streams=streams, fail=fail)
    sch = serve.Scheduler(ex, clock=clk, keep_states=True, **kw)
    m = sch.run(reqs)
    return sch, ex, m


def test_every_request_runs_exactly_its_steps():
    reqs = _trace()
    sch, ex, m = _run(reqs)
    assert m["requests"] == len(reqs)
    for r in reqs:
        assert r.steps_done == r.steps
        assert sch.states[r.id][0] == r.steps          # frozen after its last step
        assert r.arrival <= r.admitted <= r.done
    assert all(c["freed"] for c in ex.created)
    assert sch.used == 0 and sch.nactive == 0


def test_slot_limit_and_memory_budget_hold():
    reqs = _trace(n=80, rate=500.0)
    sch, ex, _ = _run(reqs, max_active=5)
    assert ex.max_live_problems <= 5
    big = max(r.nbytes for r in reqs)
    reqs2 = _trace(n=80, rate=500.0)
    sch2, ex2, _ = _run(reqs2, hbm_budget=2.5 * big)
    assert ex2.max_live_bytes <= 2.5 * big
    assert ex2.max_live_problems < len(reqs2)          # the budget made requests wait
    assert all(r.steps_done == r.steps for r in reqs2)


def test_first_come_first_served():
    reqs = _trace(n=50, rate=1000.0)
    _run(reqs, max_active=3)
    order = sorted(reqs, key=lambda r: r.arrival)
    adm = [r.admitted for r in order]
    assert all(a <= b for a, b in zip(adm, adm[1:]))


def test_cohorts_group_same_pde_and_degree():
    reqs = _trace(n=40, rate=5000.0)
    sch, ex, _ = _run(reqs)
    for c in ex.created:
        assert len({(s["pde"], s["N"]) for s in c["specs"]}) == 1
    # a burst is admitted in few passes, so several cohorts hold more than one request
    assert max(len(c["specs"]) for c in ex.created) > 1


def test_oversized_request_is_rejected():
    r = serve.Request(id=0, arrival=0.0, pde="euler", N=5, ncells=10_000, steps=3)
    sch = serve.Scheduler(FakeExecutor(VirtualClock()), hbm_budget=r.nbytes - 1)
    with pytest.raises(ValueError):
        sch.submit(r)


def test_latency_summary_is_consistent():
    reqs = _trace(n=30)
    _, _, m = _run(reqs)
    assert m["latency_ms"]["p50"] <= m["latency_ms"]["p99"]
    assert m["queue_ms"]["p50"] >= 0.0
    assert m["dof_updates_per_s"] > 0


def test_cohorts_overlap_on_the_streams():
    """Arrivals admitted while other cohorts run start at once: several
    cohorts have work on the (simulated) device at the same time."""
    reqs = _trace(n=60, rate=400.0)
    sch, ex, m = _run(reqs, streams=4)
    assert m["max_cohorts_in_flight"] >= 2
    one = _trace(n=60, rate=400.0)
    _, _, m1 = _run(one, streams=1)
    # overlapping streams finish the same trace sooner than one stream
    assert m["makespan_s"] < m1["makespan_s"]


def test_status_of_an_earlier_chunk_is_not_lost():
    """A problem that reported an error in a chunk before its last one is still
    reported when it finishes (the executor's status is sticky)."""
    reqs = [serve.Request(id=i, arrival=0.0, pde="euler", N=3, ncells=2000, steps=40) for i in range(3)]
    sch, _, _ = _run(reqs, fail={(0, 1, 0): -4}, max_steps_per_tick=10)
    assert sch.bad == {1: -4}
