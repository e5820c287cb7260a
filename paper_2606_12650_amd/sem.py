"""PyTorch-facing wrappers of libsem: device memory and streams come from
torch, every computation runs in the library's HIP kernels.

Names follow the C ABI: :class:`SemOperator` owns a ``sem_ctx`` and its
workspace; :meth:`SemOperator.ax` is ``sem_ax``, :meth:`SemOperator.cg` is
``sem_cg``; :func:`vec_axpy` and :func:`vec_dot` are the vector calls.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

LOCAL, ASSEMBLED, MASKED = L.SEM_AX_LOCAL, L.SEM_AX_ASSEMBLED, L.SEM_AX_MASKED
_PREC = {None: L.SEM_F64, "f64": L.SEM_F64, "f32": L.SEM_F32, "bf16": L.SEM_BF16}


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _check_vec(t: torch.Tensor, n: int, name: str, device) -> None:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} entries (has {t.numel()})")
    if t.device != torch.device(device):
        raise ValueError(f"{name} is on {t.device}, operator on {device}")


@dataclass
class CgResult:
    iters: int
    outer_iters: int
    status: int
    rel_res: float


def _flags(mfma) -> int:
    """None: the default kernel per order; True / False: force the matrix-core
    or the vector-ALU element kernel."""
    return 0 if mfma is None else (L.SEM_FLAG_MFMA if mfma else L.SEM_FLAG_VALU)


def mesh_desc(nelx, nely, nelz, order, deform_amp=0.0, lowprec=None, mfma=None) -> L.SemMeshDesc:
    return L.SemMeshDesc(int(nelx), int(nely), int(nelz), int(order), float(deform_amp),
                         _PREC[lowprec], _flags(mfma))


def workspace_bytes(nelx, nely, nelz, order, deform_amp=0.0, lowprec=None, mfma=None) -> int:
    d = mesh_desc(nelx, nely, nelz, order, deform_amp, lowprec, mfma)
    return int(L.lib().sem_workspace_bytes(ctypes.byref(d)))


class SemOperator:
    """The Poisson operator of one box mesh, set up on the GPU (``sem_setup``)."""

    def __init__(self, nelx, nely, nelz, order, deform_amp=0.0, lowprec=None, device="cuda", mfma=None):
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("SemOperator needs a CUDA (HIP) device")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        lib = L.lib()
        self.desc = mesh_desc(nelx, nely, nelz, order, deform_amp, lowprec, mfma)
        nbytes = int(lib.sem_workspace_bytes(ctypes.byref(self.desc)))
        if nbytes == 0:
            # the set-up's own check names the reason (SEM_ERR_ARG or SEM_ERR_UNSUPPORTED)
            rc = lib.sem_setup(ctypes.byref(self.desc), None, 0, None, ctypes.byref(ctypes.c_void_p()))
            L.check("sem_setup", rc)
            raise ValueError(f"invalid mesh descriptor {nelx}x{nely}x{nelz} N={order}")
        self.ws_bytes = nbytes
        # 256 extra bytes so the workspace can be aligned to 256.
        self._ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws_raw.data_ptr()) % 256
        self.ws = self._ws_raw[off:off + nbytes]
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check("sem_setup", lib.sem_setup(ctypes.byref(self.desc), _ptr(self.ws), nbytes,
                                               _stream(self.device), ctypes.byref(self._ctx)))
        self.nelx, self.nely, self.nelz, self.order = int(nelx), int(nely), int(nelz), int(order)
        self.E = self.nelx * self.nely * self.nelz
        self.n = self.order + 1
        self.L = int(lib.sem_nlocal(self._ctx))
        self._dot_ws = None

    def close(self) -> None:
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            L.lib().sem_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self) -> torch.Tensor:
        return torch.empty(self.L, dtype=torch.float64, device=self.device)

    def ax(self, u: torch.Tensor, mode: int = MASKED, out: torch.Tensor | None = None) -> torch.Tensor:
        """``sem_ax``: A_L u, Q Q^T A_L u or mask o Q Q^T A_L u."""
        _check_vec(u, self.L, "u", self.device)
        w = self.empty() if out is None else out
        _check_vec(w, self.L, "out", self.device)
        L.check("sem_ax", L.lib().sem_ax(self._ctx, _ptr(u), _ptr(w), int(mode), _stream(self.device)))
        return w

    def ax_lowp(self, u: torch.Tensor, mode: int = MASKED, out: torch.Tensor | None = None) -> torch.Tensor:
        """``sem_ax_lowp``: the low-precision operator on FP32 vectors."""
        if u.dtype != torch.float32 or not u.is_cuda or not u.is_contiguous() or u.numel() != self.L:
            raise ValueError("u must be a contiguous float32 CUDA tensor with L entries")
        w = torch.empty(self.L, dtype=torch.float32, device=self.device) if out is None else out
        if w.dtype != torch.float32 or w.numel() != self.L or not w.is_contiguous():
            raise ValueError("out must be a contiguous float32 tensor with L entries")
        L.check("sem_ax_lowp", L.lib().sem_ax_lowp(self._ctx, _ptr(u), _ptr(w), int(mode),
                                                   _stream(self.device)))
        return w

    def cg(self, b: torch.Tensor, x: torch.Tensor | None = None, rtol: float = 1e-8,
           max_iter: int = 0, fixed_iter: int = 0, check_every: int = 0, mixed: bool = False,
           inner_rtol: float = 0.0, inner_max: int = 0, raise_on_fail: bool = True,
           precond: bool = True):
        """``sem_cg``: Jacobi-PCG from x = 0 (``precond=False``: plain CG).
        Returns (x, CgResult)."""
        _check_vec(b, self.L, "b", self.device)
        x = self.empty() if x is None else x
        _check_vec(x, self.L, "x", self.device)
        opts = L.SemCgOpts(float(rtol), int(max_iter), int(fixed_iter), int(bool(mixed)),
                           int(check_every), float(inner_rtol), int(inner_max),
                           L.SEM_PRECOND_JACOBI if precond else L.SEM_PRECOND_NONE)
        info = L.SemCgInfo()
        rc = L.lib().sem_cg(self._ctx, _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(info),
                            _stream(self.device))
        res = CgResult(info.iters, info.outer_iters, info.status, info.rel_res)
        if rc != L.SEM_OK and (raise_on_fail or rc not in (L.SEM_ERR_NOTCONV, L.SEM_ERR_BREAKDOWN)):
            L.check("sem_cg", rc)
        return x, res

    def set_knob(self, knob: int, value: int, prec: str = "f64") -> None:
        """``sem_set_knob``: kernel variant `value` of `knob` (``OP_TILE`` or
        ``UPDATE_TILE``) for the FP64 family (``prec="f64"``) or the inner
        low-precision one (the context's ``lowprec``)."""
        L.check("sem_set_knob", L.lib().sem_set_knob(self._ctx, _PREC[prec], int(knob), int(value)))

    def get_knob(self, knob: int, prec: str = "f64") -> int:
        v = ctypes.c_int(0)
        L.check("sem_get_knob", L.lib().sem_get_knob(self._ctx, _PREC[prec], int(knob), ctypes.byref(v)))
        return v.value

    def ax_generic(self, u: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """``sem_ax_generic``: w = A_L u with the run-time-order kernel (the
        non-specialised form of the specialisation study)."""
        _check_vec(u, self.L, "u", self.device)
        w = self.empty() if out is None else out
        _check_vec(w, self.L, "out", self.device)
        L.check("sem_ax_generic", L.lib().sem_ax_generic(self._ctx, _ptr(u), _ptr(w), _stream(self.device)))
        return w

    def export(self, field: int) -> torch.Tensor:
        """``sem_export``: a copy of a setup field."""
        n1 = self.n
        size = {L.SEM_FIELD_G: 6 * self.L, L.SEM_FIELD_MINV: self.L, L.SEM_FIELD_D: n1 * n1,
                L.SEM_FIELD_NODES: 2 * n1, L.SEM_FIELD_C: self.L}[field]
        out = torch.empty(size, dtype=torch.float64, device=self.device)
        L.check("sem_export", L.lib().sem_export(self._ctx, int(field), _ptr(out), _stream(self.device)))
        return out


def vec_axpy(alpha: float, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """``vec_axpy``: y <- alpha x + y (in place)."""
    n = y.numel()
    _check_vec(x, n, "x", y.device)
    _check_vec(y, n, "y", y.device)
    L.check("vec_axpy", L.lib().vec_axpy(n, float(alpha), _ptr(x), _ptr(y), _stream(y.device)))
    return y


def gs_csr_build(gid) -> tuple[torch.Tensor, torch.Tensor]:
    """``sem_gs_csr_build``: compressed rows (offsets, ids; int32 CPU tensors)
    of the ids in ``gid`` (host int64 array or tensor) that occur at least
    twice."""
    g = torch.as_tensor(gid, dtype=torch.int64).reshape(-1).contiguous().cpu()
    n = g.numel()
    rows, copies = ctypes.c_int32(0), ctypes.c_int64(0)
    lib = L.lib()
    L.check("sem_gs_csr_build", lib.sem_gs_csr_build(n, _ptr(g), None, 0, None, 0,
                                                     ctypes.byref(rows), ctypes.byref(copies)))
    offsets = torch.empty(rows.value + 1, dtype=torch.int32)
    ids = torch.empty(max(copies.value, 1), dtype=torch.int32)
    L.check("sem_gs_csr_build", lib.sem_gs_csr_build(n, _ptr(g), _ptr(offsets), offsets.numel(),
                                                     _ptr(ids), ids.numel(), ctypes.byref(rows),
                                                     ctypes.byref(copies)))
    return offsets, ids[:copies.value]


def gs(offsets: torch.Tensor, ids: torch.Tensor, w: torch.Tensor, check: bool = True) -> torch.Tensor:
    """``sem_gs``: in place, every copy of a row of (offsets, ids) receives the
    sum of the row's copies.  offsets and ids are int32 tensors on w's device.
    ``check`` compares offsets[-1] with ids.numel() (a device read; callers
    timing repeated calls on checked rows pass False)."""
    n = w.numel()
    _check_vec(w, n, "w", w.device)
    for t, name in ((offsets, "offsets"), (ids, "ids")):
        if t.dtype != torch.int32 or t.device != w.device or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous int32 tensor on {w.device}")
    n_rows = offsets.numel() - 1
    if n_rows < 0:
        raise ValueError("offsets must hold n_rows + 1 entries")
    n_copies = ids.numel()
    if check and int(offsets[-1].item()) != n_copies:
        raise ValueError(f"ids holds {n_copies} entries but offsets[-1] = {int(offsets[-1].item())}")
    L.check("sem_gs", L.lib().sem_gs(n_rows, _ptr(offsets), _ptr(ids), n_copies, n, _ptr(w),
                                     _stream(w.device)))
    return w


def vec_dot_workspace(n: int, device) -> torch.Tensor:
    nbytes = int(L.lib().vec_dot_workspace_bytes(int(n)))
    return torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=device)


def vec_dot(x: torch.Tensor, y: torch.Tensor, wt: torch.Tensor | None = None,
            out: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """``vec_dot``: sum_i (wt_i) x_i y_i into a one-element device tensor."""
    n = x.numel()
    _check_vec(x, n, "x", x.device)
    _check_vec(y, n, "y", x.device)
    if wt is not None:
        _check_vec(wt, n, "wt", x.device)
    out = torch.empty(1, dtype=torch.float64, device=x.device) if out is None else out
    ws = vec_dot_workspace(n, x.device) if ws is None else ws
    L.check("vec_dot", L.lib().vec_dot(n, _ptr(x), _ptr(y), _ptr(wt), _ptr(out), _ptr(ws),
                                       ws.numel() * ws.element_size(), _stream(x.device)))
    return out


def vec_dot_noalloc(x: torch.Tensor, y: torch.Tensor, wt: torch.Tensor | None = None,
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """``vec_dot_noalloc``: ``vec_dot`` with the library's own partials array
    (no workspace; the output tensor is the caller's)."""
    n = x.numel()
    _check_vec(x, n, "x", x.device)
    _check_vec(y, n, "y", x.device)
    if wt is not None:
        _check_vec(wt, n, "wt", x.device)
    out = torch.empty(1, dtype=torch.float64, device=x.device) if out is None else out
    L.check("vec_dot_noalloc", L.lib().vec_dot_noalloc(n, _ptr(x), _ptr(y), _ptr(wt), _ptr(out),
                                                       _stream(x.device)))
    return out


def vec_axpy_generic(alpha: float, x: torch.Tensor, y: torch.Tensor, block: int = 256) -> torch.Tensor:
    """``vec_axpy_generic``: y <- alpha x + y with the work-group size chosen at launch."""
    n = y.numel()
    _check_vec(x, n, "x", y.device)
    _check_vec(y, n, "y", y.device)
    L.check("vec_axpy_generic", L.lib().vec_axpy_generic(n, float(alpha), _ptr(x), _ptr(y), int(block),
                                                         _stream(y.device)))
    return y


def vec_dot_generic(x: torch.Tensor, y: torch.Tensor, wt: torch.Tensor | None = None,
                    out: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                    block: int = 256) -> torch.Tensor:
    """``vec_dot_generic``: the dot with a run-time work-group size and a looped tree."""
    n = x.numel()
    _check_vec(x, n, "x", x.device)
    _check_vec(y, n, "y", x.device)
    if wt is not None:
        _check_vec(wt, n, "wt", x.device)
    out = torch.empty(1, dtype=torch.float64, device=x.device) if out is None else out
    if ws is None:
        nbytes = int(L.lib().vec_dot_generic_workspace_bytes(int(n), int(block)))
        ws = torch.empty(max(1, (nbytes + 7) // 8), dtype=torch.float64, device=x.device)
    L.check("vec_dot_generic", L.lib().vec_dot_generic(n, _ptr(x), _ptr(y), _ptr(wt), _ptr(out), _ptr(ws),
                                                       ws.numel() * ws.element_size(), int(block),
                                                       _stream(x.device)))
    return out


OP_TILE, UPDATE_TILE = L.SEM_KNOB_OP_TILE, L.SEM_KNOB_UPDATE_TILE


def knob_count(order: int, knob: int, prec: str = "f64") -> int:
    """``sem_knob_count``: candidates of a knob for an order and precision family."""
    return int(L.lib().sem_knob_count(int(order), _PREC[prec], int(knob)))
