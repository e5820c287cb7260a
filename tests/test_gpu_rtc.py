"""Orders 13..15: the per-order kernels compiled at set-up with hipRTC (the
jit-clause analogue), against the FP64 oracle through the C ABI.

Bars as for the built orders: setup fields 1e-13, A.u (local, assembled,
masked) max|dw| <= 1e-12 max|w_ref|, 20 fixed CG iterations (Jacobi and
plain) ||dx||_c / ||x_ref||_c <= 1e-9, x bitwise continuous across copies.
"""

import math
import os
import time

import numpy as np
import pytest
import torch

import workload
from oracle import operator as op, pcg as opcg

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


def _rel_inf(a, ref):
    return float(np.max(np.abs(a - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _c_norm(v, c):
    return math.sqrt(float(np.sum(c.reshape(-1) * v.reshape(-1) ** 2)))


def _same_on_copies(pr, v):
    gid = pr.gid.reshape(-1)
    hi = np.full(gid.max() + 1, -np.inf)
    lo = np.full(gid.max() + 1, np.inf)
    np.maximum.at(hi, gid, v.reshape(-1))
    np.minimum.at(lo, gid, v.reshape(-1))
    return bool(np.array_equal(hi, lo))


@pytest.mark.parametrize("N", [13, 14, 15])
def test_rtc_order_setup_ax_and_cg(N):
    mesh = (3, 2, 2)
    amp = 0.05
    pr = op.Problem(*mesh, N, amp)
    t0 = time.perf_counter()
    A = sem.SemOperator(*mesh, N, amp, device=DEV)
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    B = sem.SemOperator(*mesh, N, amp, device=DEV)
    t_again = time.perf_counter() - t0
    print(f"[rtc] N={N}: first set-up (compile and load) {t_first:.2f} s, again {t_again:.3f} s", flush=True)
    # setup fields
    G = _cpu(A.export(L.SEM_FIELD_G)).reshape(pr.G.shape)
    assert _rel_inf(G, pr.G) <= 1e-13
    minv = _cpu(A.export(L.SEM_FIELD_MINV)).reshape(pr.minv.shape)
    assert _rel_inf(minv, pr.minv) <= 1e-13
    c = _cpu(A.export(L.SEM_FIELD_C)).reshape(pr.c.shape)
    assert np.array_equal(c, pr.c)
    # A.u in the three modes
    u_disc = workload.iid_lvector(300 + N, pr.L)
    u_cont = workload.continuous_rhs(400 + N, *mesh, N, zero_boundary=False)
    w = _cpu(A.ax(_gpu(u_disc), sem.LOCAL)).reshape(pr.mask.shape)
    assert _rel_inf(w, pr.ax_local(u_disc)) <= 1e-12
    w = _cpu(A.ax(_gpu(u_cont), sem.ASSEMBLED)).reshape(pr.mask.shape)
    assert _rel_inf(w, pr.ax_assembled(u_cont)) <= 1e-12
    w = _cpu(A.ax(_gpu(u_cont), sem.MASKED)).reshape(pr.mask.shape)
    assert _rel_inf(w, pr.ax(u_cont)) <= 1e-12
    assert np.all(w[pr.mask == 0] == 0.0)
    # CG: 20 fixed iterations, Jacobi and plain
    b = workload.continuous_rhs(500 + N, *mesh, N)
    for precond, minv_or in ((True, pr.minv), (False, pr.mask)):
        xr, info = opcg.pcg(pr.ax, pr.shape4(b), minv_or, pr.c, fixed_iter=20)
        xg, res = A.cg(_gpu(b), fixed_iter=20, precond=precond)
        assert res.iters == 20 and res.status == 0
        x = _cpu(xg)
        assert _c_norm(x - xr.reshape(-1), pr.c) / _c_norm(xr, pr.c) <= 1e-9, precond
        assert abs(res.rel_res - info["rel_res"]) <= 1e-6 * info["rel_res"]
        assert _same_on_copies(pr, x)
    # the second operator (kernels from the process cache) gives the same bits
    x1, _ = A.cg(_gpu(b), fixed_iter=20)
    x2, _ = B.cg(_gpu(b), fixed_iter=20)
    assert torch.equal(x1, x2)
    A.close()
    B.close()


@pytest.mark.parametrize("N", [13, 15])
def test_rtc_order_tolerance_mode_and_ragged_mesh(N):
    mesh = (2, 3, 1)
    pr = op.Problem(*mesh, N, 0.05)
    A = sem.SemOperator(*mesh, N, 0.05, device=DEV, mfma=True)
    b = workload.continuous_rhs(600 + N, *mesh, N)
    xr, info = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, rtol=1e-8)
    xg, res = A.cg(_gpu(b), rtol=1e-8, check_every=7)
    assert res.status == 0 and abs(res.iters - info["iters"]) <= 2
    tr = opcg.true_rel_residual(pr.ax, pr.shape4(b), pr.shape4(_cpu(xg)), pr.c)
    assert tr <= 1e-8 * (1 + 1e-3)
    A.close()


def test_rtc_order_refuses_low_precision_and_vector_tile():
    for kw in ({"lowprec": "f32"}, {"mfma": False}):
        with pytest.raises(sem.SemError) as ex:
            sem.SemOperator(2, 2, 2, 13, 0.0, device=DEV, **kw)
        assert ex.value.code == L.SEM_ERR_UNSUPPORTED
