"""ctypes binding of libsem.so (declarations mirror include/sem.h).

Only argument marshalling lives here; every step of the computation runs in
the library's HIP kernels.  Loading fails loudly when the library is missing.
"""

from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsem.so")

SEM_OK = 0
SEM_ERR_ARG = -1
SEM_ERR_HIP = -2
SEM_ERR_NOMEM = -3
SEM_ERR_NOTCONV = -4
SEM_ERR_BREAKDOWN = -5
SEM_ERR_UNSUPPORTED = -6

SEM_F64, SEM_F32, SEM_BF16 = 0, 1, 2
SEM_AX_LOCAL, SEM_AX_ASSEMBLED, SEM_AX_MASKED = 0, 1, 3
SEM_FIELD_G, SEM_FIELD_MINV, SEM_FIELD_D, SEM_FIELD_NODES, SEM_FIELD_C = 0, 1, 2, 3, 4
SEM_FLAG_MFMA, SEM_FLAG_VALU = 1, 2
SEM_PRECOND_JACOBI, SEM_PRECOND_NONE = 0, 1
SEM_KNOB_OP_TILE, SEM_KNOB_UPDATE_TILE = 0, 1

# Every symbol include/sem.h declares.
EXPORTS = (
    "sem_workspace_bytes", "sem_setup", "sem_destroy", "sem_nlocal", "sem_ax", "sem_cg",
    "vec_axpy", "vec_dot_workspace_bytes", "vec_dot", "sem_export", "sem_last_error",
    "sem_ax_lowp", "sem_batch_workspace_bytes", "sem_batch_create", "sem_batch_set_tile",
    "sem_batch_add", "sem_batch_step", "sem_batch_poll", "sem_batch_remove", "sem_batch_destroy",
    "sem_gs_csr_build", "sem_gs", "vec_dot_noalloc", "sem_rtc_build",
    "sem_ax_generic", "vec_axpy_generic", "vec_dot_generic_workspace_bytes", "vec_dot_generic",
    "sem_knob_count", "sem_set_knob", "sem_get_knob",
)


class SemMeshDesc(ctypes.Structure):
    _fields_ = [("nelx", ctypes.c_int32), ("nely", ctypes.c_int32), ("nelz", ctypes.c_int32),
                ("order", ctypes.c_int32), ("deform_amp", ctypes.c_double),
                ("lowprec", ctypes.c_int32), ("flags", ctypes.c_int32)]


class SemCgOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("fixed_iter", ctypes.c_int32), ("mixed", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("inner_max", ctypes.c_int32), ("precond", ctypes.c_int32)]


class SemCgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("rel_res", ctypes.c_double)]


class SemError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


_lib = None


def _declare(lib):
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "sem_workspace_bytes": (sz, [P(SemMeshDesc)]),
        "sem_setup": (ctypes.c_int, [P(SemMeshDesc), vp, sz, vp, P(vp)]),
        "sem_destroy": (ctypes.c_int, [vp]),
        "sem_nlocal": (i64, [vp]),
        "sem_ax": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp]),
        "sem_ax_lowp": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, vp]),
        "sem_cg": (ctypes.c_int, [vp, vp, vp, P(SemCgOpts), P(SemCgInfo), vp]),
        "vec_axpy": (ctypes.c_int, [i64, dbl, vp, vp, vp]),
        "vec_dot_workspace_bytes": (sz, [i64]),
        "vec_dot": (ctypes.c_int, [i64, vp, vp, vp, vp, vp, sz, vp]),
        "sem_export": (ctypes.c_int, [vp, ctypes.c_int, vp, vp]),
        "sem_last_error": (ctypes.c_char_p, []),
        "sem_batch_workspace_bytes": (sz, [ctypes.c_int]),
        "sem_batch_create": (ctypes.c_int, [ctypes.c_int, vp, sz, vp, P(vp)]),
        "sem_batch_set_tile": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "sem_batch_add": (ctypes.c_int, [vp, vp, vp, vp, P(SemCgOpts), P(ctypes.c_int), vp]),
        "sem_batch_step": (ctypes.c_int, [vp, ctypes.c_int, vp]),
        "sem_batch_poll": (ctypes.c_int, [vp, P(ctypes.c_int), ctypes.c_int, P(ctypes.c_int),
                                          P(SemCgInfo), P(ctypes.c_int), vp]),
        "sem_batch_remove": (ctypes.c_int, [vp, ctypes.c_int, vp]),
        "sem_batch_destroy": (ctypes.c_int, [vp]),
        "sem_gs_csr_build": (ctypes.c_int, [i64, vp, vp, i64, vp, i64, P(i32), P(i64)]),
        "sem_gs": (ctypes.c_int, [i32, vp, vp, i64, i64, vp, vp]),
        "vec_dot_noalloc": (ctypes.c_int, [i64, vp, vp, vp, vp, vp]),
        "sem_rtc_build": (ctypes.c_int, [ctypes.c_int, ctypes.c_char_p, P(sz)]),
        "sem_ax_generic": (ctypes.c_int, [vp, vp, vp, vp]),
        "sem_knob_count": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "sem_set_knob": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "sem_get_knob": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, P(ctypes.c_int)]),
        "vec_axpy_generic": (ctypes.c_int, [i64, dbl, vp, vp, ctypes.c_int, vp]),
        "vec_dot_generic_workspace_bytes": (sz, [i64, ctypes.c_int]),
        "vec_dot_generic": (ctypes.c_int, [i64, vp, vp, vp, vp, vp, sz, ctypes.c_int, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    del i32


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsem.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        handle = ctypes.CDLL(LIB_PATH)
        _declare(handle)
        _lib = handle
    return _lib


def check(fn: str, code: int) -> int:
    if code != SEM_OK:
        raise SemError(fn, code, lib().sem_last_error().decode())
    return code
