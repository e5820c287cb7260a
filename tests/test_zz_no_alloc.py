"""vec_dot_noalloc (the dot product for callers that cannot allocate) against
vec_dot, both called through the C ABI on the same device data.

Both run the same kernels in the same summation order, so the bar is bitwise
equality; the first call is also held to the dot tolerance against the
exactly rounded value (|dot - exact| <= 1e-13 sum|w_i x_i y_i|).  Two calls
follow each other, the second on a smaller input, so the library's shared
partials array still holds the first call's larger set of partials when the
second runs.
"""

import ctypes
import os

import numpy as np
import pytest
import torch

from oracle.dots import abs_sum, dot_exact

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
MAX_N = 65536 * 2048  # the array's capacity in vector entries


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"[gpu-test] {os.environ.get('PYTEST_CURRENT_TEST', '')}", flush=True)


def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _dots(lib, x, y, wt):
    """(vec_dot, vec_dot_noalloc) of the same data on the current stream."""
    from paper_2606_12650_amd import _lib as L

    n = x.numel()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    nbytes = int(lib.vec_dot_workspace_bytes(n))
    ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=DEV)
    ref = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    got = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    assert lib.vec_dot(n, _p(x), _p(y), _p(wt), _p(ref), _p(ws), nbytes, s) == L.SEM_OK
    rc = lib.vec_dot_noalloc(n, _p(x), _p(y), _p(wt), _p(got), s)
    assert rc == L.SEM_OK, lib.sem_last_error()
    torch.cuda.synchronize()
    return float(ref.item()), float(got.item())


def test_noalloc_equals_vec_dot_two_calls_second_smaller():
    from paper_2606_12650_amd import _lib as L

    lib = L.lib()
    rng = np.random.default_rng(77)
    # first call: weighted, several thousand tiles and a ragged last tile
    n1 = 5_000_003
    x1, y1, w1 = (rng.uniform(-1.0, 1.0, n1) for _ in range(3))
    w1 = np.abs(w1)
    tx, ty, tw = (torch.from_numpy(a).to(DEV) for a in (x1, y1, w1))
    ref1, got1 = _dots(lib, tx, ty, tw)
    assert got1 == ref1  # bitwise: same kernels, same order
    exact1 = dot_exact(x1, y1, w1)
    assert abs(got1 - exact1) <= 1e-13 * abs_sum(x1, y1, w1)
    # second call: smaller, unweighted
    n2 = 70_001
    x2, y2 = rng.uniform(-1.0, 1.0, n2), rng.uniform(-1.0, 1.0, n2)
    ref2, got2 = _dots(lib, torch.from_numpy(x2).to(DEV), torch.from_numpy(y2).to(DEV), None)
    assert got2 == ref2
    assert abs(got2 - dot_exact(x2, y2)) <= 1e-13 * abs_sum(x2, y2)
    # empty vector: 0, and the array's old contents do not leak in
    _, got0 = _dots(lib, torch.empty(0, dtype=torch.float64, device=DEV),
                    torch.empty(0, dtype=torch.float64, device=DEV), None)
    assert got0 == 0.0


def test_noalloc_at_capacity_and_refusal_beyond():
    from paper_2606_12650_amd import _lib as L

    lib = L.lib()
    g = torch.Generator(device=DEV)
    g.manual_seed(5)
    x = torch.rand(MAX_N, generator=g, dtype=torch.float64, device=DEV) - 0.5
    y = torch.rand(MAX_N, generator=g, dtype=torch.float64, device=DEV) - 0.5
    ref, got = _dots(lib, x, y, None)
    assert got == ref
    # then a smaller one on the same array
    ref_s, got_s = _dots(lib, x[:123457], y[:123457], None)
    assert got_s == ref_s
    out = torch.zeros(1, dtype=torch.float64, device=DEV)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.vec_dot_noalloc(MAX_N + 1, _p(x), _p(y), None, _p(out), s) == L.SEM_ERR_ARG
    assert b"exceeds" in lib.sem_last_error()
    torch.cuda.synchronize()
    assert out.item() == 0.0  # nothing was enqueued
