"""GPU parity of every compiled kernel variant the tuning knobs select
(sem_set_knob): each candidate CG update tile shape and element tile, per
order, in FP64 against the oracle and in the mixed-precision solver against
the FP64 oracle solution.

Tolerances as for the default kernels:
  FP64 CG, 20 fixed iterations   ||x_gpu - x_ref||_c / ||x_ref||_c <= 1e-9
  mixed CG to 1e-8               FP64 true residual <= 1e-8 (1 + 1e-3) and
                                 ||x - x_ref||_c / ||x_ref||_c <= 1e-5
and x stays bitwise equal on every copy of a shared node (the update sums a
node's copies in the same order on every copy, in every tile shape).
"""

import math
import os

import numpy as np
import pytest
import torch

import workload
from oracle import operator as op
from oracle import pcg as opcg

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


def _mesh(N):
    # several update tiles of every candidate shape (up to 128 elements per
    # tile at N = 1) and a ragged last tile
    if N <= 3:
        return 8, 7, 6
    if N <= 8:
        return 5, 4, 3
    return 3, 2, 3


def _same_on_copies(pr, v):
    gid = pr.gid.reshape(-1)
    flat = np.asarray(v).reshape(-1)
    order = np.argsort(gid, kind="stable")
    g, f = gid[order], flat[order]
    first = np.r_[True, g[1:] != g[:-1]]
    lead = np.maximum.accumulate(np.where(first, np.arange(g.size), 0))
    return bool(np.array_equal(f, f[lead]))


def _crel(pr, a, ref):
    c = pr.c.reshape(-1)
    d = a.reshape(-1) - ref.reshape(-1)
    return math.sqrt(float(np.sum(c * d * d)) / float(np.sum(c * ref.reshape(-1) ** 2)))


@pytest.mark.parametrize("N", list(range(1, 13)))
def test_update_tile_variants_fp64_match_oracle(N):
    nx, ny, nz = _mesh(N)
    amp = 0.05
    pr = op.Problem(nx, ny, nz, N, amp)
    bnp = workload.continuous_rhs(40 + N, nx, ny, nz, N)
    xr, _ = opcg.pcg(pr.ax, pr.shape4(bnp), pr.minv, pr.c, fixed_iter=20)
    A = sem.SemOperator(nx, ny, nz, N, amp, device=DEV)
    b = torch.from_numpy(bnp).to(DEV)
    nvar = sem.knob_count(N, sem.UPDATE_TILE)
    assert nvar == 4
    for v in range(nvar):
        A.set_knob(sem.UPDATE_TILE, v)
        assert A.get_knob(sem.UPDATE_TILE) == v
        x, res = A.cg(b, fixed_iter=20)
        torch.cuda.synchronize()
        xg = x.cpu().numpy()
        assert res.iters == 20
        rel = _crel(pr, xg, xr)
        assert rel <= 1e-9, (N, v, rel)
        assert _same_on_copies(pr, xg), (N, v)
    A.close()


@pytest.mark.parametrize("N", [1, 3, 5, 7, 9, 10, 11, 12])
@pytest.mark.parametrize("lowprec", ["f32", "bf16"])
def test_inner_update_tile_variants_mixed_solve(N, lowprec):
    nx, ny, nz = _mesh(N)
    amp = 0.05
    pr = op.Problem(nx, ny, nz, N, amp)
    bnp = workload.continuous_rhs(60 + N, nx, ny, nz, N)
    b4 = pr.shape4(bnp)
    xr, info = opcg.pcg(pr.ax, b4, pr.minv, pr.c, rtol=1e-12)
    assert info["converged"]
    A = sem.SemOperator(nx, ny, nz, N, amp, lowprec=lowprec, device=DEV)
    b = torch.from_numpy(bnp).to(DEV)
    for v in range(sem.knob_count(N, sem.UPDATE_TILE, lowprec)):
        A.set_knob(sem.UPDATE_TILE, v, lowprec)
        x, res = A.cg(b, rtol=1e-8, mixed=True)
        assert res.status == 0, (N, lowprec, v)
        torch.cuda.synchronize()
        xg = x.cpu().numpy()
        tr = opcg.true_rel_residual(pr.ax, b4, pr.shape4(xg), pr.c)
        assert tr <= 1e-8 * (1 + 1e-3), (N, lowprec, v, tr)
        assert _crel(pr, xg, xr) <= 1e-5, (N, lowprec, v)
    A.close()


@pytest.mark.parametrize("N", [3, 7, 11])
def test_op_tile_knob_matches_oracle(N):
    nx, ny, nz = 3, 2, 3
    amp = 0.05
    pr = op.Problem(nx, ny, nz, N, amp)
    u = workload.continuous_rhs(70 + N, nx, ny, nz, N)
    ref = pr.ax(u).reshape(-1)
    A = sem.SemOperator(nx, ny, nz, N, amp, device=DEV)
    ug = torch.from_numpy(u).to(DEV)
    assert sem.knob_count(N, sem.OP_TILE) == 3
    outs = []
    for v in range(3):
        A.set_knob(sem.OP_TILE, v)
        w = A.ax(ug, sem.MASKED)
        torch.cuda.synchronize()
        wg = w.cpu().numpy()
        assert np.max(np.abs(wg - ref)) <= 1e-12 * np.max(np.abs(ref))
        outs.append(wg)
    # the default is one of the two tiles, bit for bit
    assert np.array_equal(outs[0], outs[1]) or np.array_equal(outs[0], outs[2])
    A.close()


def test_knob_errors_and_batch_refusal():
    A = sem.SemOperator(2, 2, 2, 5, 0.0, device=DEV)
    for bad in (-1, 4, 99):
        with pytest.raises(L.SemError) as ei:
            A.set_knob(sem.UPDATE_TILE, bad)
        assert ei.value.code == L.SEM_ERR_UNSUPPORTED
    with pytest.raises(L.SemError):
        A.set_knob(7, 0)
    with pytest.raises(L.SemError):
        A.set_knob(sem.UPDATE_TILE, 0, "f32")  # no low-precision copy
    assert sem.knob_count(13, sem.UPDATE_TILE) == 1
    assert sem.knob_count(13, sem.OP_TILE) == 1
    assert sem.knob_count(13, sem.UPDATE_TILE, "f32") == 0
    assert sem.knob_count(0, sem.UPDATE_TILE) == 0
    A.set_knob(sem.UPDATE_TILE, 2)
    from paper_2606_12650_amd.batch import SemBatch
    B = SemBatch(2, device=DEV)
    b = torch.zeros(A.L, dtype=torch.float64, device=DEV)
    with pytest.raises(L.SemError):
        B.add(A, b)
    A.set_knob(sem.UPDATE_TILE, 0)
    slot = B.add(A, b)  # defaults again: accepted
    B.remove(slot)
    B.close()
    A.close()
