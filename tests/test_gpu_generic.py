"""GPU parity of the non-specialised kernels of the specialisation study
(run-time order N, run-time work-group size, looped in-group reduction;
paper Sec. VIII-B, Tab. hip_vs_hip) against the FP64 oracle, and against the
specialised kernels they are timed beside.

Tolerances as for the specialised kernels:
  A_L u      max|w_gpu - w_ref| <= 1e-12 * max|w_ref|
  dots       |dot_gpu - dot_exact| <= 1e-13 * sum|x_i y_i w_i|
  axpy       |y_gpu - y_ref| <= 2^-52 * (|y| + |alpha x|) elementwise
"""

import os

import numpy as np
import pytest
import torch

import workload
from oracle import operator as op
from oracle.dots import abs_sum, dot_exact

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2606_12650_amd as sem
    from paper_2606_12650_amd import _lib as L

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"[gpu-test] {os.environ.get('PYTEST_CURRENT_TEST', '')}", flush=True)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to(DEV)


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("N", list(range(1, 12)))
def test_ax_generic_matches_oracle(N):
    nx, ny, nz, amp = 3, 2, 3, 0.05  # 18 elements: several work-groups and a ragged last one
    pr = op.Problem(nx, ny, nz, N, amp)
    A = sem.SemOperator(nx, ny, nz, N, amp, device=DEV)
    u = workload.iid_lvector(20 + N, A.L)
    w = _cpu(A.ax_generic(_gpu(u))).reshape(pr.shape4(u).shape)
    ref = pr.ax_local(u)
    assert np.max(np.abs(w - ref)) <= 1e-12 * np.max(np.abs(ref))
    # the specialised vector-ALU tile computes the same sums
    Av = sem.SemOperator(nx, ny, nz, N, amp, device=DEV, mfma=False)
    wv = _cpu(Av.ax(_gpu(u), sem.LOCAL)).reshape(w.shape)
    assert np.max(np.abs(w - wv)) <= 1e-12 * np.max(np.abs(ref))
    A.close()
    Av.close()


def test_ax_generic_refuses_order_12():
    A = sem.SemOperator(2, 2, 2, 12, 0.0, device=DEV)
    u = torch.zeros(A.L, dtype=torch.float64, device=DEV)
    with pytest.raises(L.SemError) as ei:
        A.ax_generic(u)
    assert ei.value.code == L.SEM_ERR_UNSUPPORTED
    A.close()


@pytest.mark.parametrize("n", [0, 1, 63, 4097, 100_003, 1_000_003])
@pytest.mark.parametrize("block", [64, 256, 1024])
def test_dot_generic_matches_exact(n, block):
    rng = np.random.default_rng(n + block)
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    wt = rng.uniform(0.1, 1, n)
    for weight in (None, wt):
        got = float(_cpu(sem.vec_dot_generic(_gpu(x), _gpu(y), None if weight is None else _gpu(weight),
                                             block=block))[0])
        ref = dot_exact(x, y, weight)
        assert abs(got - ref) <= 1e-13 * max(abs_sum(x, y, weight), 1e-300)
    # deterministic for fixed (n, block)
    a = _cpu(sem.vec_dot_generic(_gpu(x), _gpu(y), block=block))
    b = _cpu(sem.vec_dot_generic(_gpu(x), _gpu(y), block=block))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [0, 5, 4097, 1_000_003])
@pytest.mark.parametrize("block", [64, 512])
def test_axpy_generic_matches_bound(n, block):
    rng = np.random.default_rng(7 + n)
    x = rng.uniform(-1, 1, n)
    y = rng.uniform(-1, 1, n)
    alpha = 0.5 + 1.0 / 3.0
    yg = _gpu(y)
    sem.vec_axpy_generic(alpha, _gpu(x), yg, block=block)
    got = _cpu(yg)
    ref = y + alpha * x
    assert np.all(np.abs(got - ref) <= 2.0 ** -52 * (np.abs(y) + np.abs(alpha * x)))
    # the specialised kernel (one FMA per entry) gives the same bits
    ys = _gpu(y)
    sem.vec_axpy(alpha, _gpu(x), ys)
    assert np.array_equal(_cpu(ys), got)


def test_generic_block_checked():
    x = torch.zeros(10, dtype=torch.float64, device=DEV)
    for bad in (0, 48, 96, 2048):
        with pytest.raises(L.SemError):
            sem.vec_axpy_generic(1.0, x, x.clone(), block=bad)
        with pytest.raises(L.SemError):
            sem.vec_dot_generic(x, x, block=bad, ws=torch.zeros(8, dtype=torch.float64, device=DEV))
