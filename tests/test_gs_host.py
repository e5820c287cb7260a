"""Host side of the generic gather-scatter: the library's compressed-row
builder (host C++, no GPU call) produces exactly the oracle's rows, and
rejects bad arguments with an error code."""

import ctypes

import numpy as np
import pytest

from oracle import gs as ogs
from paper_2606_12650_amd import _lib as L
from paper_2606_12650_amd import sem


@pytest.mark.parametrize("case", ["random", "periodic", "box", "unique", "one_id"])
def test_csr_build_matches_oracle(case):
    rng = np.random.default_rng(11)
    if case == "random":
        gid = rng.integers(0, 700, 2000)
    elif case == "periodic":
        gid = ogs.periodic_global_ids(3, 2, 2, 4)
    elif case == "box":
        gid = ogs.periodic_global_ids(2, 3, 2, 5, periodic=(False, False, False))
    elif case == "unique":
        gid = rng.permutation(500)
    else:
        gid = np.full(40, 12345)
    off, ids = sem.gs_csr_build(gid)
    o_off, o_ids = ogs.csr_from_ids(gid)
    assert off.numpy().tolist() == o_off.tolist()
    assert ids.numpy().tolist() == o_ids.tolist()


def test_csr_build_errors():
    lib = L.lib()
    rows, copies = ctypes.c_int32(0), ctypes.c_int64(0)
    g = np.array([0, 1, -3], dtype=np.int64)
    rc = lib.sem_gs_csr_build(3, g.ctypes.data, None, 0, None, 0, ctypes.byref(rows), ctypes.byref(copies))
    assert rc == L.SEM_ERR_ARG
    g = np.array([4, 4, 5, 5, 5], dtype=np.int64)
    rc = lib.sem_gs_csr_build(5, g.ctypes.data, None, 0, None, 0, ctypes.byref(rows), ctypes.byref(copies))
    assert rc == L.SEM_OK and rows.value == 2 and copies.value == 5
    off = np.zeros(3, dtype=np.int32)
    ids = np.zeros(4, dtype=np.int32)  # one short
    rc = lib.sem_gs_csr_build(5, g.ctypes.data, off.ctypes.data, 3, ids.ctypes.data, 4,
                              ctypes.byref(rows), ctypes.byref(copies))
    assert rc == L.SEM_ERR_NOMEM
    rc = lib.sem_gs_csr_build(-1, g.ctypes.data, None, 0, None, 0, ctypes.byref(rows), ctypes.byref(copies))
    assert rc == L.SEM_ERR_ARG
    # empty input: no rows
    rc = lib.sem_gs_csr_build(0, None, None, 0, None, 0, ctypes.byref(rows), ctypes.byref(copies))
    assert rc == L.SEM_OK and rows.value == 0 and copies.value == 0


def test_gs_rejects_bad_sizes_before_launch():
    lib = L.lib()
    assert lib.sem_gs(-1, None, None, 0, 0, None, None) == L.SEM_ERR_ARG
    assert lib.sem_gs(3, None, None, 0, 10, None, None) == L.SEM_ERR_ARG
    assert lib.sem_gs(0, None, None, 0, -1, None, None) == L.SEM_ERR_ARG
    assert lib.sem_gs(0, None, None, -1, 0, None, None) == L.SEM_ERR_ARG
