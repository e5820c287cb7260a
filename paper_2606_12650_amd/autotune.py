"""Tile-shape autotuner for the batched operator kernel.

For each polynomial order and arithmetic, the batched persistent kernel can
process operator work items of several sizes (elements per 256-thread
work-group; the compiled set is probed through ``sem_batch_set_tile``).  The
tuner times each candidate on the device with a small batch of solves of that
order and keeps the fastest.  Results are cached in JSON keyed by the device
context, in the spirit of the paper's transformation scripts that pick launch
shapes from device parameters (Sec. V-B, Tab. context_params: device name,
vendor, driver, backend, maximum threads per block).
"""

from __future__ import annotations

import json
import os
import time

import torch

from . import _lib as L
from .batch import SemBatch
from .sem import SemOperator

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
