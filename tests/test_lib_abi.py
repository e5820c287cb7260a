"""The C-ABI library loads, exports every declared symbol and validates its
arguments on the host (no GPU work is launched by these tests)."""

import ctypes
import os
import re

import pytest

from paper_2606_12650_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "sem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) - {"sizeof"})


def test_header_and_binding_agree():
    assert _declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_symbol():
    lib = L.lib()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_workspace_bytes_host_only():
    lib = L.lib()
    d = L.SemMeshDesc(32, 32, 32, 7, 0.05, 0, 0)
    nb = lib.sem_workspace_bytes(ctypes.byref(d))
    Lpts = 32768 * 512
    # G (6) + Minv + r + p + w = 10 doubles per point, plus small buffers
    assert 80 * Lpts <= nb < 80 * Lpts + 4 * 2 ** 20
    bad = L.SemMeshDesc(0, 1, 1, 7, 0.0, 0, 0)
    assert lib.sem_workspace_bytes(ctypes.byref(bad)) == 0
    bad = L.SemMeshDesc(1, 1, 1, 16, 0.0, 0, 0)  # above the run-time compiled orders 13..15
    assert lib.sem_workspace_bytes(ctypes.byref(bad)) == 0
    # the 32-bit index arithmetic caps a mesh at 4e9 element-local points
    big = L.SemMeshDesc(193, 193, 193, 7, 0.0, 0, 0)  # 3.68e9 points
    assert lib.sem_workspace_bytes(ctypes.byref(big)) > 80 * 193 ** 3 * 512
    for n, N in ((200, 7), (100, 15), (256, 12)):  # 4.1e9, 4.1e9, 3.7e10 points
        bad = L.SemMeshDesc(n, n, n, N, 0.0, 0, 0)
        assert lib.sem_workspace_bytes(ctypes.byref(bad)) == 0
    # unknown flag bits are refused; the matrix-core flag costs no memory
    for flags in (3, 4, -1):
        bad = L.SemMeshDesc(2, 2, 2, 7, 0.0, L.SEM_F32, flags)
        assert lib.sem_workspace_bytes(ctypes.byref(bad)) == 0
    ok = L.SemMeshDesc(2, 2, 2, 7, 0.0, L.SEM_BF16, L.SEM_FLAG_MFMA)
    plain = L.SemMeshDesc(2, 2, 2, 7, 0.0, L.SEM_BF16, 0)
    assert lib.sem_workspace_bytes(ctypes.byref(ok)) == lib.sem_workspace_bytes(ctypes.byref(plain)) > 0
    f64 = L.SemMeshDesc(2, 2, 2, 7, 0.0, L.SEM_F64, L.SEM_FLAG_MFMA)
    assert lib.sem_workspace_bytes(ctypes.byref(f64)) == lib.sem_workspace_bytes(
        ctypes.byref(L.SemMeshDesc(2, 2, 2, 7, 0.0, L.SEM_F64, 0)))


def test_argument_errors_return_codes_without_launching():
    lib = L.lib()
    d = L.SemMeshDesc(2, 2, 2, 3, 0.0, 0, 0)
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: checks fail first
    assert lib.sem_setup(None, fake, 1 << 30, None, ctypes.byref(ctx)) == L.SEM_ERR_ARG
    assert lib.sem_setup(ctypes.byref(d), None, 1 << 30, None, ctypes.byref(ctx)) == L.SEM_ERR_ARG
    assert lib.sem_setup(ctypes.byref(d), ctypes.c_void_p((1 << 20) + 8), 1 << 30, None,
                         ctypes.byref(ctx)) == L.SEM_ERR_ARG
    assert lib.sem_setup(ctypes.byref(d), fake, 16, None, ctypes.byref(ctx)) == L.SEM_ERR_NOMEM
    assert b"needs" in lib.sem_last_error()
    assert lib.sem_ax(None, fake, fake, 3, None) == L.SEM_ERR_ARG
    assert lib.vec_axpy(-1, 1.0, None, None, None) == L.SEM_ERR_ARG
    assert lib.vec_dot(5, None, None, None, fake, fake, 1024, None) == L.SEM_ERR_ARG
    assert lib.vec_dot(5, fake, fake, None, fake, fake, 0, None) == L.SEM_ERR_NOMEM
    assert lib.sem_nlocal(None) == -1
    assert lib.sem_destroy(None) == L.SEM_ERR_ARG
    assert lib.vec_dot_workspace_bytes(2049) == 16
    # vec_dot_noalloc refuses negative and over-capacity lengths before any HIP call
    assert lib.vec_dot_noalloc(-1, fake, fake, None, fake, None) == L.SEM_ERR_ARG
    assert lib.vec_dot_noalloc(65536 * 2048 + 1, fake, fake, None, fake, None) == L.SEM_ERR_ARG
    assert b"exceeds" in lib.sem_last_error()
    assert lib.vec_dot_noalloc(4, None, fake, None, fake, None) == L.SEM_ERR_ARG
    assert lib.vec_dot_noalloc(4, fake, fake, None, None, None) == L.SEM_ERR_ARG


def test_batch_workspace_and_create_arguments_host_only():
    lib = L.lib()
    assert lib.sem_batch_workspace_bytes(0) == 0
    assert lib.sem_batch_workspace_bytes(4097) == 0
    one, many = lib.sem_batch_workspace_bytes(1), lib.sem_batch_workspace_bytes(256)
    assert 0 < one < many
    h = ctypes.c_void_p()
    assert lib.sem_batch_create(0, None, 0, None, ctypes.byref(h)) == L.SEM_ERR_ARG
    assert lib.sem_batch_create(4, None, many, None, ctypes.byref(h)) == L.SEM_ERR_ARG
    assert not h.value

