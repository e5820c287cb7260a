"""Autotuners for the kernel shapes.

``tune`` (batches): for each polynomial order and arithmetic, the batched
persistent kernel can process operator work items of several sizes
(elements per work-group; the compiled set is probed through
``sem_batch_set_tile``); the tuner times each candidate with a small batch of
solves of that order and keeps the fastest.

``tune_solver`` (single solves): for each order and precision family, the
element operator's tile (matrix-core or vector-ALU) and the CG update tile's
shape (threads per column, elements per tile, plane ranges) are compiled in
several candidates (``sem_knob_count``); the tuner times CG iterations with
each on a mesh of the given size and keeps the fastest of each knob.

Results are cached in JSON keyed by the device context, in the spirit of the
paper's transformation scripts that pick launch shapes from device
parameters (Sec. V-B, Tab. context_params: device name, vendor, driver,
backend, maximum threads per block).
"""

from __future__ import annotations

import json
import os
import time

import torch

from . import _lib as L
from .batch import SemBatch
from .sem import OP_TILE, UPDATE_TILE, SemOperator, knob_count

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sem_mi355x", "tiles.json")
CANDIDATES = range(1, 65)


def context(device) -> dict:
    dev = torch.device(device)
    p = torch.cuda.get_device_properties(dev)
    return {
        "device::name": p.name,
        "device::arch": getattr(p, "gcnArchName", ""),
        "device::vendor": "AMD",
        "device::driver": str(torch.version.hip),
        "device::max_threads_per_block": 1024,
        "backend::name": "HIP",
    }


def _key(ctx: dict, prec: str, order: int) -> str:
    return f"{ctx['device::name']}|{ctx['device::arch']}|{ctx['device::driver']}|{prec}|N{order}"


_PREC_CODE = {"f64": L.SEM_F64, "f32": L.SEM_F32, "bf16": L.SEM_BF16}


def supported_tiles(order: int, device, prec: str = "f64") -> list[int]:
    B = SemBatch(1, device=device)
    out = []
    for epb in CANDIDATES:
        if L.lib().sem_batch_set_tile(B._h, _PREC_CODE[prec], int(order), int(epb)) == L.SEM_OK:
            out.append(epb)
    B.close()
    return out


def _time_tile(order: int, epb: int, prec: str, device, nel: int, instances: int, iters: int) -> float:
    lowprec = None if prec == "f64" else prec
    ops, bs = [], []
    for i in range(instances):
        op = SemOperator(nel, nel, nel, order, 0.05, lowprec=lowprec, device=device)
        b = torch.ones(op.L, dtype=torch.float64, device=device)
        ops.append(op)
        bs.append(b)
    B = SemBatch(instances, device=device)
    B.set_tile(order, epb, "f64" if lowprec is None else lowprec)
    for op, b in zip(ops, bs):
        # a tolerance no solve reaches in the timed steps: every step does full work
        B.add(op, b, rtol=1e-30, mixed=lowprec is not None, max_iter=10 ** 6, inner_max=10 ** 6)
    B.step(iters)  # warm-up and graph capture
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    B.step(iters)
    torch.cuda.synchronize(device)
    dt = time.perf_counter() - t0
    B.close()
    for op in ops:
        op.close()
    return dt / iters


def tune(orders=(3, 5, 7, 9, 11), precisions=("f64", "f32", "bf16"), device="cuda", elements=None,
         instances=4, iters=20, cache_path: str | None = DEFAULT_CACHE, refresh=False) -> dict:
    """Best elements-per-item for each (precision, order); cached by context."""
    dev = torch.device(device)
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    ctx = context(dev)
    cache = {}
    if cache_path and os.path.exists(cache_path) and not refresh:
        with open(cache_path) as fh:
            cache = json.load(fh)
    out: dict = {p: {} for p in precisions}
    timings: dict = {}
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        for prec in precisions:
            for order in orders:
                key = _key(ctx, prec, order)
                if key in cache:
                    out[prec][order] = int(cache[key]["epb"])
                    continue
                nel = elements or max(4, int(round((12000.0 / (order + 1) ** 3) ** (1 / 3) * 4)))
                best, best_t = None, float("inf")
                for epb in supported_tiles(order, dev, prec):
                    t = _time_tile(order, epb, prec, dev, nel, instances, iters)
                    timings[(prec, order, epb)] = t
                    if t < best_t:
                        best, best_t = epb, t
                out[prec][order] = best
                cache[key] = {"epb": best, "us_per_step": best_t * 1e6,
                              "candidates": {str(e): timings[(prec, order, e)] * 1e6
                                             for (p, o, e) in timings if p == prec and o == order}}
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return out


def apply(batch: SemBatch, tiles: dict, precs=("f64", "f32", "bf16")) -> None:
    """Set the tuned tiles of the given precisions on a batch."""
    for prec in precs:
        for order, epb in tiles.get(prec, {}).items():
            if epb:
                batch.set_tile(int(order), int(epb), prec)


def _time_iters(op: SemOperator, b: torch.Tensor, x: torch.Tensor, prec: str, iters: int, reps: int) -> float:
    """Seconds per CG iteration of the family `prec`: FP64 Jacobi-PCG for
    ``f64``; for ``f32`` / ``bf16`` one outer step of the mixed solver whose
    inner solve runs exactly `iters` iterations (an inner tolerance it never
    reaches), so the inner operator and update dominate.  Best of `reps`."""
    best = float("inf")
    for r in range(reps + 1):
        torch.cuda.synchronize(op.device)
        t0 = time.perf_counter()
        if prec == "f64":
            op.cg(b, x, fixed_iter=iters, check_every=iters)
        else:
            op.cg(b, x, rtol=1e-30, mixed=True, max_iter=1, inner_rtol=1e-30, inner_max=iters,
                  check_every=iters, raise_on_fail=False)
        torch.cuda.synchronize(op.device)
        if r > 0:  # the first run captures the graph
            best = min(best, time.perf_counter() - t0)
    return best / iters


def tune_solver(orders=(7, 11), precisions=("f64", "f32", "bf16"), device="cuda", box=(32, 32, 32),
                iters=100, reps=3, cache_path: str | None = DEFAULT_CACHE, refresh=False) -> dict:
    """Fastest element tile and CG update tile per (precision family, order).

    Returns {prec: {order: {"op_tile": v, "update_tile": v, "us_per_iter": t,
    "op_tile_us": {v: t}, "update_tile_us": {v: t}}}}: the element tile is
    chosen first with the default update tile, then the update tile with the
    chosen element tile.  Times are microseconds per CG iteration on the
    deformed box `box` (for the mixed families: per inner iteration plus a
    share of one outer step)."""
    dev = torch.device(device)
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    ctx = context(dev)
    cache = {}
    if cache_path and os.path.exists(cache_path) and not refresh:
        with open(cache_path) as fh:
            cache = json.load(fh)
    out: dict = {p: {} for p in precisions}
    nx, ny, nz = box
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        for order in orders:
            b = None
            for prec in precisions:
                key = _key(ctx, prec, order) + f"|solver|{nx}x{ny}x{nz}"
                if key in cache:
                    out[prec][order] = cache[key]
                    continue
                op = SemOperator(nx, ny, nz, order, 0.05, lowprec=None if prec == "f64" else prec, device=dev)
                if b is None or b.numel() != op.L:
                    b = torch.ones(op.L, dtype=torch.float64, device=dev)
                x = torch.empty_like(b)
                res = {"op_tile_us": {}, "update_tile_us": {}}
                for v in (1, 2):  # matrix-core, vector-ALU (0, the default, is one of them)
                    op.set_knob(OP_TILE, v, prec)
                    res["op_tile_us"][v] = _time_iters(op, b, x, prec, iters, reps) * 1e6
                best_op = min(res["op_tile_us"], key=res["op_tile_us"].get)
                op.set_knob(OP_TILE, best_op, prec)
                for v in range(knob_count(order, UPDATE_TILE, prec)):
                    op.set_knob(UPDATE_TILE, v, prec)
                    res["update_tile_us"][v] = _time_iters(op, b, x, prec, iters, reps) * 1e6
                best_up = min(res["update_tile_us"], key=res["update_tile_us"].get)
                res.update(op_tile=best_op, update_tile=best_up, us_per_iter=res["update_tile_us"][best_up])
                op.close()
                out[prec][order] = res
                cache[key] = res
            del b
    torch.cuda.synchronize(dev)
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return out


def apply_solver(op: SemOperator, tuned: dict, precs=("f64",)) -> None:
    """Set the tuned knobs of `op`'s order on it (for the listed families)."""
    for prec in precs:
        r = tuned.get(prec, {}).get(op.order) or tuned.get(prec, {}).get(str(op.order))
        if r:
            op.set_knob(OP_TILE, int(r["op_tile"]), prec)
            op.set_knob(UPDATE_TILE, int(r["update_tile"]), prec)
