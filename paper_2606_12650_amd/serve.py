"""Serving form: continuous batching of Poisson-arrival solve requests.

Requests (a box mesh, an order, a seeded right-hand side) arrive over time.
The scheduler admits them first-come first-served while a batch slot is free
and their device footprint (``sem_workspace_bytes`` plus b and x) fits the
HBM budget; every step advances all admitted solves by a few CG iterations in
one batched launch sequence; finished solves leave at once and free their
slot and memory for the next request.  Requests that arrive while others are
on the GPU therefore join the running batch (iteration-level continuous
batching), not a queue behind it.

The policy (:class:`Scheduler`) is separate from the device work
(:class:`GpuExecutor`) so that it can be exercised with a simulated clock.
The baseline :func:`serve_per_request` solves one request at a time with
``sem_cg`` in FP64.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    index: int
    nx: int
    ny: int
    nz: int
    N: int
    amp: float
    rhs_seed: int
    arrival: float  # seconds from the start of the run

    @property
    def E(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def L(self) -> int:
        return self.E * (self.N + 1) ** 3


@dataclass
class Completion:
    index: int
    arrival: float
    admitted: float
    finished: float
    iters: int
    outer_iters: int
    status: int
    rel_res: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class ServeStats:
    completions: list = field(default_factory=list)
    rejected: list = field(default_factory=list)
    wall: float = 0.0
    max_active: int = 0
    peak_bytes: int = 0
    gpu_busy_s: float = 0.0  # time the batch stream spent in batched steps (GPU executor)

    def summary(self, warmup: int = 0) -> dict:
        """Latency percentiles and throughput over the requests after the
        first ``warmup`` (in arrival order).  Throughput counts the timed
        requests that converged, over the window from the first timed
        arrival to the last timed completion."""
        done = sorted(self.completions, key=lambda c: c.arrival)
        timed = done[warmup:] if warmup < len(done) else []
        lat = np.array([c.latency for c in timed]) if timed else np.zeros(1)
        ok = sum(1 for c in timed if c.status == 0)
        window = (max(c.finished for c in timed) - min(c.arrival for c in timed)) if timed else 0.0
        return {
            "requests": len(self.completions) + len(self.rejected),
            "completed": len(self.completions),
            "converged": sum(1 for c in self.completions if c.status == 0),
            "rejected": len(self.rejected),
            "warmup": min(warmup, len(done)),
            "timed": len(timed),
            "solves_per_s": ok / window if window > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()),
            "wall_s": self.wall,
            "max_active": self.max_active,
            "peak_bytes": self.peak_bytes,
            "gpu_busy_frac": self.gpu_busy_s / self.wall if self.wall > 0 else 0.0,
        }


def make_requests(specs: list[dict], arrivals) -> list[Request]:
    return [Request(s["index"], s["nx"], s["ny"], s["nz"], s["N"], s["amp"], s["rhs_seed"], float(t))
            for s, t in zip(specs, arrivals)]


class Scheduler:
    """First-come first-served admission by free slot and HBM budget, with
    iteration-level continuous batching.

    ``executor`` provides ``footprint(req)``, ``admit(req) -> slot``,
    ``step()``, ``poll() -> [(slot, result)]``, ``release(slot)`` and
    ``active``; ``clock()`` returns seconds since the start and
    ``sleep(dt)`` waits (both injectable for tests).

    An executor that also provides ``prepare(req) -> token``,
    ``admit_prepared(token) -> slot`` and ``launch_step()`` (asynchronous,
    finished by ``poll``) gets admission off the device's critical path: the
    expensive part of admitting (set-up of the operator and the right-hand
    side) runs while the batched step of the admitted requests is on the
    GPU, and only the cheap insertion of prepared requests into the batch
    happens between steps.  A prepared request holds its slot and memory.
    With ``step_done() -> bool`` as well, set-ups stop once the running step
    has ended (after at least one), so a burst of arrivals does not leave
    the device idle while the host prepares it.
    """

    def __init__(self, executor, hbm_budget: int, max_slots: int, clock=None, sleep=None):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        t0 = time.perf_counter()
        self.clock = clock or (lambda: time.perf_counter() - t0)
        self.sleep = sleep or time.sleep

    def run(self, requests: list[Request]) -> ServeStats:
        if all(hasattr(self.ex, a) for a in ("prepare", "admit_prepared", "launch_step")):
            return self._run_overlapped(requests)
        stats = ServeStats()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue: deque = deque()
        active: dict = {}  # slot -> (request, footprint, admitted time)
        used = 0
        start = self.clock()
        while pending or queue or active:
            now = self.clock()
            while pending and pending[0].arrival <= now - start:
                queue.append(pending.popleft())
            while queue and len(active) < self.max_slots:
                req = queue[0]
                fp = self.ex.footprint(req)
                if fp > self.budget:  # can never fit: refuse rather than block the queue
                    queue.popleft()
                    stats.rejected.append(req.index)
                    continue
                if used + fp > self.budget:
                    break
                queue.popleft()
                slot = self.ex.admit(req)
                active[slot] = (req, fp, self.clock() - start)
                used += fp
                stats.peak_bytes = max(stats.peak_bytes, used)
            stats.max_active = max(stats.max_active, len(active))
            if active:
                self.ex.step()
                done = self.ex.poll()
                tnow = self.clock() - start
                for slot, res in done:
                    req, fp, adm = active.pop(slot)
                    self.ex.release(slot)
                    used -= fp
                    stats.completions.append(Completion(req.index, req.arrival, adm, tnow, res.iters,
                                                        res.outer_iters, res.status, res.rel_res))
            elif pending:
                wait = pending[0].arrival - (self.clock() - start)
                if wait > 0:
                    self.sleep(wait)
        stats.wall = self.clock() - start
        stats.gpu_busy_s = getattr(self.ex, "busy_s", 0.0)
        return stats

    def _run_overlapped(self, requests: list[Request]) -> ServeStats:
        stats = ServeStats()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        queue: deque = deque()
        prepared: deque = deque()  # (request, token, footprint, admitted time)
        active: dict = {}  # slot -> (request, footprint, admitted time)
        used = 0
        start = self.clock()

        def take_arrivals():
            now = self.clock() - start
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())

        step_done = getattr(self.ex, "step_done", None)

        def prepare_queued(boxed: bool):
            # boxed: stop once the device is free (the running step has
            # ended, or none runs) so that the next step does not wait for
            # set-ups; one set-up always goes ahead, so admission keeps moving
            nonlocal used
            n = 0
            while queue and len(active) + len(prepared) < self.max_slots:
                if boxed and n > 0 and step_done is not None and step_done():
                    break
                req = queue[0]
                fp = self.ex.footprint(req)
                if fp > self.budget:  # can never fit: refuse rather than block the queue
                    queue.popleft()
                    stats.rejected.append(req.index)
                    continue
                if used + fp > self.budget:
                    break
                queue.popleft()
                adm = self.clock() - start
                prepared.append((req, self.ex.prepare(req), fp, adm))
                n += 1
                used += fp
                stats.peak_bytes = max(stats.peak_bytes, used)

        while pending or queue or prepared or active:
            take_arrivals()
            if not active and not prepared:
                prepare_queued(boxed=True)  # nothing on the device: start it soon
            while prepared:
                req, token, fp, adm = prepared.popleft()
                active[self.ex.admit_prepared(token)] = (req, fp, adm)
            stats.max_active = max(stats.max_active, len(active))
            if active:
                self.ex.launch_step()
                # the step runs on the device: admit what has arrived meanwhile
                take_arrivals()
                prepare_queued(boxed=True)
                done = self.ex.poll()
                tnow = self.clock() - start
                for slot, res in done:
                    req, fp, adm = active.pop(slot)
                    self.ex.release(slot)
                    used -= fp
                    stats.completions.append(Completion(req.index, req.arrival, adm, tnow, res.iters,
                                                        res.outer_iters, res.status, res.rel_res))
            elif pending and not queue and not prepared:
                wait = pending[0].arrival - (self.clock() - start)
                if wait > 0:
                    self.sleep(wait)
        stats.wall = self.clock() - start
        stats.gpu_busy_s = getattr(self.ex, "busy_s", 0.0)
        return stats


class GpuExecutor:
    """Device side of the scheduler: one SemBatch on the batch stream; each
    admitted request gets its own SemOperator and a right-hand side drawn on
    the GPU from its seed, both made on a side stream while the batched step
    runs (``prepare``), then joined to the batch between steps
    (``admit_prepared``).  HIP events around every step measure the time the
    batch stream is busy."""

    def __init__(self, device="cuda", max_slots=64, mixed: str | None = "f32", iters_per_step=10,
                 tiles: dict | None = None,
                 rtol=1e-8, keep_solutions=False):
        import torch

        from .batch import SemBatch

        self.torch = torch
        self.device = torch.device(device)
        self.mixed = mixed
        self.iters = int(iters_per_step)
        self.rtol = rtol
        self.stream = torch.cuda.current_stream(self.device)  # the batch stream
        self.setup_stream = torch.cuda.Stream(device=self.device)
        self.batch = SemBatch(max_slots, device=self.device)
        for prec, per_order in (tiles or {}).items():  # {"f64" / "f32" / "bf16": {order: epb}}
            for order, epb in per_order.items():
                self.batch.set_tile(int(order), int(epb), prec)
        self.slots: dict = {}
        self.keep = keep_solutions
        self.solutions: dict = {}  # request index -> x (when keep_solutions)
        self.busy_s = 0.0
        self._events = None

    def footprint(self, req: Request) -> int:
        from .sem import workspace_bytes

        return workspace_bytes(req.nx, req.ny, req.nz, req.N, req.amp, self.mixed) + 16 * req.L + 512

    def prepare(self, req: Request):
        """Set up the request's operator and right-hand side on the side
        stream (sem_setup waits for that stream only)."""
        import workload

        from .sem import SemOperator

        torch = self.torch
        with torch.cuda.stream(self.setup_stream):
            op = SemOperator(req.nx, req.ny, req.nz, req.N, req.amp, lowprec=self.mixed, device=self.device)
            b = workload.continuous_rhs_device(req.rhs_seed, req.nx, req.ny, req.nz, req.N, self.device)
        self.setup_stream.synchronize()
        # the batch stream uses these from now on
        op._ws_raw.record_stream(self.stream)
        b.record_stream(self.stream)
        return req, op, b

    def admit_prepared(self, token) -> int:
        req, op, b = token
        slot = self.batch.add(op, b, rtol=self.rtol, mixed=self.mixed is not None)
        self.slots[slot] = req
        return slot

    def admit(self, req: Request) -> int:
        return self.admit_prepared(self.prepare(req))

    def launch_step(self) -> None:
        torch = self.torch
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        self.batch.step(self.iters)
        e1.record(self.stream)
        self._events = (e0, e1)

    def step(self) -> None:
        self.launch_step()

    def step_done(self) -> bool:
        """The launched step has finished on the device (no wait)."""
        return self._events is None or self._events[1].query()

    def poll(self):
        fin, _ = self.batch.poll()  # waits for the step
        if self._events is not None:
            self.busy_s += self._events[0].elapsed_time(self._events[1]) / 1e3
            self._events = None
        return fin

    def release(self, slot: int):
        op, b, x = self.batch.remove(slot)
        req = self.slots.pop(slot, None)
        op.close()
        if self.keep and req is not None:
            self.solutions[req.index] = x
        return x

    @property
    def active(self) -> int:
        return len(self.slots)


def serve_per_request(requests: list[Request], device="cuda", rtol=1e-8, clock=None,
                      sleep=None) -> ServeStats:
    """Baseline: one request at a time, FP64 ``sem_cg``, in arrival order."""
    import torch

    import workload

    from .sem import SemOperator

    t0 = time.perf_counter()
    clock = clock or (lambda: time.perf_counter() - t0)
    sleep = sleep or time.sleep
    stats = ServeStats()
    dev = torch.device(device)
    stream = torch.cuda.Stream(device=dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(stream):
        start = clock()
        for req in sorted(requests, key=lambda r: r.arrival):
            wait = req.arrival - (clock() - start)
            if wait > 0:
                sleep(wait)
            adm = clock() - start
            op = SemOperator(req.nx, req.ny, req.nz, req.N, req.amp, device=dev)
            b = workload.continuous_rhs_device(req.rhs_seed, req.nx, req.ny, req.nz, req.N, dev)
            _, res = op.cg(b, rtol=rtol, raise_on_fail=False)
            op.close()
            stats.completions.append(Completion(req.index, req.arrival, adm, clock() - start, res.iters,
                                                res.outer_iters, res.status, res.rel_res))
            stats.max_active = 1
        stats.wall = clock() - start
    torch.cuda.synchronize(dev)
    return stats


def serve(requests: list[Request], device="cuda", mixed: str | None = "f32", hbm_budget=32 << 30,
          max_slots=64, iters_per_step=10, tiles: dict | None = None, rtol=1e-8,
          keep_solutions=False):
    """Run the continuous-batching server over ``requests`` on one GPU, on a
    stream of its own (so that each batched step replays as one graph).
    Returns (ServeStats, {request index: x} or {})."""
    import torch

    dev = torch.device(device)
    stream = torch.cuda.Stream(device=dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(stream):
        ex = GpuExecutor(dev, max_slots=max_slots, mixed=mixed, iters_per_step=iters_per_step,
                         tiles=tiles, rtol=rtol, keep_solutions=keep_solutions)
        try:
            stats = Scheduler(ex, hbm_budget, max_slots).run(requests)
        finally:
            ex.batch.close()
    torch.cuda.synchronize(dev)
    return stats, ex.solutions
