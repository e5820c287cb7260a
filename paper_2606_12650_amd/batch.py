"""Batched and continuously batched solves (the ``sem_batch_*`` C ABI).

:class:`SemBatch` owns a ``sem_batch`` and its workspace.  Solves (each a
:class:`~paper_2606_12650_amd.sem.SemOperator` with a right-hand side) join
free slots, every :meth:`SemBatch.step` advances all of them by CG
iterations in one captured graph, and :meth:`SemBatch.poll` reports the ones
that finished.  All computation runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes
import math

import torch

from . import _lib as L
from .sem import CgResult, SemOperator, _check_vec, _ptr, _stream

VEC_TILE = 2048  # entries per streaming item
_PREC_CODE = {"f64": L.SEM_F64, "f32": L.SEM_F32, "bf16": L.SEM_BF16}


def items_for(op: SemOperator, epb: int) -> tuple[int, int]:
    """(operator items, vector items) a solve on ``op`` gives each iteration."""
    return math.ceil(op.E / epb), math.ceil(op.L / VEC_TILE)


def default_epb(order: int, prec: str = "f64") -> int:
    """The library's default elements per operator item (the single-solve tile
    of the element kernel that order and precision run by default)."""
    n1 = order + 1
    if order >= {"f64": 7, "f32": 7, "bf16": 9}[prec]:  # matrix-core tile
        nt = (n1 * n1 + 15) // 16  # column tiles; waves per element: a multiple of four above two
        nw = nt if nt <= 2 else (16 if nt > 8 else (nt + 3) // 4 * 4)
        return 1 if nw >= 8 else 8 // nw
    return 1 if n1 * n1 >= 128 else 128 // (n1 * n1)


class SemBatch:
    def __init__(self, max_slots: int, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        lib = L.lib()
        nbytes = int(lib.sem_batch_workspace_bytes(int(max_slots)))
        if nbytes == 0:
            raise ValueError("max_slots must be in 1..4096")
        self._ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws_raw.data_ptr()) % 256
        self.ws = self._ws_raw[off:off + nbytes]
        self._h = ctypes.c_void_p()
        L.check("sem_batch_create", lib.sem_batch_create(int(max_slots), _ptr(self.ws), nbytes,
                                                          _stream(self.device), ctypes.byref(self._h)))
        self.max_slots = int(max_slots)
        self._slots: dict[int, tuple] = {}
        self._fin = (ctypes.c_int * self.max_slots)()
        self._infos = (L.SemCgInfo * self.max_slots)()

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().sem_batch_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._slots.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile(self, order: int, elements_per_item: int, prec: str = "f64") -> None:
        """Elements per operator item of one order for FP64 work ("f64") or the
        inner iterations of mixed solves ("f32", "bf16")."""
        L.check("sem_batch_set_tile", L.lib().sem_batch_set_tile(self._h, _PREC_CODE[prec], int(order),
                                                                  int(elements_per_item)))

    def add(self, op: SemOperator, b: torch.Tensor, x: torch.Tensor | None = None, rtol: float = 1e-8,
            mixed: bool = False, max_iter: int = 0, inner_rtol: float = 0.0, inner_max: int = 0) -> int:
        """Start a solve in a free slot; returns the slot index."""
        x = op.empty() if x is None else x
        _check_vec(b, op.L, "b", op.device)
        _check_vec(x, op.L, "x", op.device)
        opts = L.SemCgOpts(float(rtol), int(max_iter), 0, int(bool(mixed)), 0, float(inner_rtol),
                           int(inner_max), 0)
        slot = ctypes.c_int(-1)
        L.check("sem_batch_add", L.lib().sem_batch_add(self._h, op._ctx, _ptr(b), _ptr(x), ctypes.byref(opts),
                                                       ctypes.byref(slot), _stream(self.device)))
        self._slots[slot.value] = (op, b, x)
        return slot.value

    def step(self, iters: int = 1) -> None:
        L.check("sem_batch_step", L.lib().sem_batch_step(self._h, int(iters), _stream(self.device)))

    def poll(self):
        """Returns ([(slot, CgResult), ...] for finished slots, active count)."""
        nf = ctypes.c_int(0)
        na = ctypes.c_int(0)
        L.check("sem_batch_poll", L.lib().sem_batch_poll(self._h, self._fin, self.max_slots, ctypes.byref(nf),
                                                         self._infos, ctypes.byref(na), _stream(self.device)))
        out = []
        for q in range(nf.value):
            i = self._infos[q]
            out.append((self._fin[q], CgResult(i.iters, i.outer_iters, i.status, i.rel_res)))
        return out, na.value

    def remove(self, slot: int):
        """Free a slot; returns (operator, b, x) of its solve."""
        L.check("sem_batch_remove", L.lib().sem_batch_remove(self._h, int(slot), _stream(self.device)))
        return self._slots.pop(slot)

    def solution(self, slot: int) -> torch.Tensor:
        return self._slots[slot][2]

    def run_all(self, iters_per_step: int = 10, max_steps: int = 100000) -> dict[int, CgResult]:
        """Step until every occupied slot has finished; returns results by slot
        (the slots stay occupied until removed)."""
        results: dict[int, CgResult] = {}
        for _ in range(max_steps):
            fin, active = self.poll()
            for slot, res in fin:
                results[slot] = res
            if len(results) >= active:
                return results
            self.step(iters_per_step)
        raise RuntimeError("batch did not finish within max_steps")
