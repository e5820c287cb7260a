"""CPU tests of the serving policy: admission by HBM budget and free slots,
first-come first-served order, iteration-level continuous batching, and
latency accounting, with a simulated clock and a stub executor (test
scaffolding; the product's executor is the GPU batch)."""

import numpy as np
import pytest

import workload
from paper_2606_12650_amd.serve import Request, Scheduler, make_requests


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class Result:
    def __init__(self, iters):
        self.iters, self.outer_iters, self.status, self.rel_res = iters, 0, 0, 1e-9


class StubExecutor:
    """Each request needs ceil(L / 5000) steps of 1 ms; one step advances every
    admitted request (what a batched step does)."""

    def __init__(self, clock, budget_per_point=100):
        self.clock = clock
        self.left = {}
        self.bpp = budget_per_point
        self.next_slot = 0
        self.free = []
        self.log = []  # (time, event, index, used)
        self.used = 0
        self.fp = {}

    def footprint(self, req):
        return req.L * self.bpp

    def admit(self, req):
        slot = self.free.pop() if self.free else self.next_slot
        if slot == self.next_slot:
            self.next_slot += 1
        self.left[slot] = (req, max(1, -(-req.L // 5000)))
        self.used += self.footprint(req)
        self.fp[slot] = self.footprint(req)
        self.log.append((self.clock(), "admit", req.index, self.used))
        return slot

    def step(self):
        self.clock.t += 1e-3
        for s in list(self.left):
            r, n = self.left[s]
            self.left[s] = (r, n - 1)

    def poll(self):
        return [(s, Result(3)) for s, (r, n) in self.left.items() if n <= 0]

    def release(self, slot):
        req, _ = self.left.pop(slot)
        self.used -= self.fp.pop(slot)
        self.free.append(slot)
        self.log.append((self.clock(), "release", req.index, self.used))


def _requests(n=60, rate=500.0, seed=5):
    specs = workload.serving_requests(seed, n, e_lo=8, e_hi=512)
    return make_requests(specs, workload.poisson_arrivals(seed, rate, n))


@pytest.mark.parametrize("budget_mult,slots", [(3e5, 4), (1e6, 16), (2e7, 64)])
def test_budget_and_slots_respected(budget_mult, slots):
    clk = Clock()
    ex = StubExecutor(clk)
    reqs = _requests()
    budget = int(budget_mult * 100)
    stats = Scheduler(ex, budget, slots, clock=clk, sleep=clk.sleep).run(reqs)
    assert len(stats.completions) + len(stats.rejected) == len(reqs)
    assert all(u <= budget for _, _, _, u in ex.log)
    assert stats.max_active <= slots
    for c in stats.completions:
        assert c.arrival <= c.admitted <= c.finished
    fits = [r.index for r in reqs if r.L * 100 <= budget]
    assert sorted(c.index for c in stats.completions) == sorted(fits)
    assert sorted(stats.rejected) == sorted(set(r.index for r in reqs) - set(fits))


def test_fifo_admission_order():
    clk = Clock()
    ex = StubExecutor(clk)
    reqs = _requests(n=40, rate=2000.0)
    Scheduler(ex, 10 ** 9, 8, clock=clk, sleep=clk.sleep).run(reqs)
    admitted = [i for _, ev, i, _ in ex.log if ev == "admit"]
    order = [r.index for r in sorted(reqs, key=lambda r: r.arrival)]
    assert admitted == order


def test_continuous_batching_joins_running_batch():
    """A short request arriving while a long one runs is admitted at once and
    finishes first (iteration-level batching, not run-to-completion)."""
    clk = Clock()
    ex = StubExecutor(clk)
    long = Request(0, 10, 10, 10, 7, 0.05, 1, 0.0)   # 512000 points: 103 steps
    short = Request(1, 2, 2, 2, 3, 0.05, 2, 0.010)   # 512 points: 1 step
    stats = Scheduler(ex, 10 ** 12, 4, clock=clk, sleep=clk.sleep).run([long, short])
    by = {c.index: c for c in stats.completions}
    assert by[1].admitted < by[0].finished
    assert by[1].finished < by[0].finished
    assert by[1].latency < 0.005


def test_latency_statistics():
    clk = Clock()
    ex = StubExecutor(clk)
    stats = Scheduler(ex, 10 ** 12, 16, clock=clk, sleep=clk.sleep).run(_requests(n=100))
    s = stats.summary()
    lat = sorted(c.latency for c in stats.completions)
    assert s["completed"] == 100 and s["converged"] == 100
    assert abs(s["p50_latency_s"] - float(np.percentile(lat, 50))) < 1e-12
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


class OverlapStub(StubExecutor):
    """The same work model, with admission split as the GPU executor splits
    it: ``prepare`` costs host time (the set-up), ``launch_step`` starts a
    1 ms device step and returns at once, ``poll`` waits for its end."""

    SETUP = 0.4e-3

    def __init__(self, clock, **kw):
        super().__init__(clock, **kw)
        self.step_end = None
        self.busy_s = 0.0

    def prepare(self, req):
        self.clock.t += self.SETUP
        return req

    def admit_prepared(self, req):
        return super().admit(req)

    def admit(self, req):  # the sequential path: set-up then insertion
        return self.admit_prepared(self.prepare(req))

    def launch_step(self):
        self.step_end = self.clock.t + 1e-3
        self.busy_s += 1e-3
        for s in list(self.left):
            r, n = self.left[s]
            self.left[s] = (r, n - 1)

    def poll(self):
        self.clock.t = max(self.clock.t, self.step_end)
        return super().poll()


class BoxedStub(OverlapStub):
    """The same, and it reports whether the launched step has ended."""

    def step_done(self):
        return self.step_end is None or self.clock.t >= self.step_end


class SequentialStub(OverlapStub):
    """Same costs, without the overlap (the executor interface of the
    sequential path only)."""


    def __getattribute__(self, name):
        if name in ("prepare", "admit_prepared", "launch_step"):
            raise AttributeError(name)
        return object.__getattribute__(self, name)

    def admit(self, req):
        self.clock.t += self.SETUP
        return StubExecutor.admit(self, req)

    def step(self):
        OverlapStub.launch_step(self)
        self.clock.t = max(self.clock.t, self.step_end)


def test_overlapped_admission_keeps_policy_and_hides_setup():
    reqs = _requests(n=80, rate=3000.0)
    results = {}
    for name, cls in (("overlap", OverlapStub), ("sequential", SequentialStub)):
        clk = Clock()
        ex = cls(clk)
        budget = int(2e6 * 100)
        stats = Scheduler(ex, budget, 8, clock=clk, sleep=clk.sleep).run(reqs)
        s = stats.summary()
        assert s["completed"] + s["rejected"] == len(reqs)
        assert all(u <= budget for _, _, _, u in ex.log)
        assert stats.max_active <= 8
        admitted = [i for _, ev, i, _ in ex.log if ev == "admit"]
        fits = [r.index for r in sorted(reqs, key=lambda r: r.arrival) if r.L * 100 <= budget]
        assert admitted == fits  # first come, first served
        results[name] = s
    # the set-ups overlap the device steps: less wall time, a busier device
    assert results["overlap"]["wall_s"] < results["sequential"]["wall_s"]
    assert results["overlap"]["gpu_busy_frac"] > results["sequential"]["gpu_busy_frac"]


def test_summary_excludes_warmup():
    clk = Clock()
    ex = StubExecutor(clk)
    reqs = _requests(n=50)
    stats = Scheduler(ex, 10 ** 12, 16, clock=clk, sleep=clk.sleep).run(reqs)
    s0, s10 = stats.summary(), stats.summary(warmup=10)
    assert s0["timed"] == 50 and s10["timed"] == 40 and s10["warmup"] == 10
    timed = sorted(stats.completions, key=lambda c: c.arrival)[10:]
    assert abs(s10["p50_latency_s"] - float(np.percentile([c.latency for c in timed], 50))) < 1e-12


def test_setups_stop_when_the_step_ends():
    """With step_done, a burst of arrivals is prepared a few set-ups per step
    (at least one) instead of all while the device waits: same admission
    order and budget, a busier device, less wall time."""
    reqs = _requests(n=120, rate=2e4)
    res = {}
    for name, cls in (("boxed", BoxedStub), ("unboxed", OverlapStub)):
        clk = Clock()
        ex = cls(clk)
        ex.SETUP = 0.6e-3  # more than half a step: two set-ups outlast it
        budget = int(4e6 * 100)
        stats = Scheduler(ex, budget, 32, clock=clk, sleep=clk.sleep).run(reqs)
        s = stats.summary()
        assert s["completed"] + s["rejected"] == len(reqs)
        assert all(u <= budget for _, _, _, u in ex.log)
        admitted = [i for _, ev, i, _ in ex.log if ev == "admit"]
        fits = [r.index for r in sorted(reqs, key=lambda r: r.arrival) if r.L * 100 <= budget]
        assert admitted == fits
        res[name] = s
    assert res["boxed"]["gpu_busy_frac"] > res["unboxed"]["gpu_busy_frac"]
    assert res["boxed"]["wall_s"] < res["unboxed"]["wall_s"]

