"""GPU parity of the precision form: the low-precision operator and the
inner-outer CG, through the C ABI, against the FP64 oracle.

Low-precision A.u (componentwise, B = |D|^T |G| |D| |u| with rounded operands,
assembled like the result):
  FP32: |w_gpu - w_ref| <= (4 (N+1) + 8) 2^-24 B   (FP32 accumulation of the
        two contractions and the 3-term metric product; w_ref evaluates the
        rounded operator in FP64)
  BF16: |w_gpu - w_ref| <= 2^-7 B   (the FP32-accumulated weighted gradient
        may round to the neighbouring bfloat16 value: one bfloat16 ulp, plus
        the FP32 accumulation)
Inner-outer CG: the solve reports an FP64 true residual <= rtol, and
||x - x_ref||_c / ||x_ref||_c <= 1e-5 against the oracle's FP64 solution
(condition number times the residual tolerance).
"""

import math
import os
import types

import numpy as np
import pytest
import torch

import workload
from oracle import operator as op, pcg as opcg
from oracle.mixed import ax_local_abs_bound, ax_local_rounded

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


def _tol(prec, N):
    return (4 * (N + 1) + 8) * 2.0 ** -24 if prec == "f32" else 2.0 ** -7


@pytest.mark.parametrize("mfma", [False, True], ids=["valu", "mfma"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("N", [1, 3, 5, 7, 9, 11, 12])
def test_lowp_operator_componentwise(prec, N, mfma):
    nx, ny, nz, amp = 3, 2, 2, 0.05
    pr = op.Problem(nx, ny, nz, N, amp)
    A = sem.SemOperator(nx, ny, nz, N, amp, lowprec=prec, device=DEV, mfma=mfma)
    u = workload.iid_lvector(300 + N, pr.L).astype(np.float32).astype(np.float64)
    ug = torch.from_numpy(u.astype(np.float32)).to(DEV)
    ref = ax_local_rounded(pr, u, prec)
    B = ax_local_abs_bound(pr, u, prec)
    w = A.ax_lowp(ug, sem.LOCAL).cpu().numpy().astype(np.float64).reshape(ref.shape)
    err = np.abs(w - ref)
    assert np.all(err <= _tol(prec, N) * B + 1e-30), float(np.max(err / (B + 1e-30)))
    # assembled and masked: the same bound, summed over copies
    refm = pr.mask * pr.dssum(ref)
    Bm = pr.dssum(B)
    wm = A.ax_lowp(ug, sem.MASKED).cpu().numpy().astype(np.float64).reshape(ref.shape)
    assert np.all(np.abs(wm - refm) <= _tol(prec, N) * Bm + 1e-30)
    assert np.all(wm[pr.mask == 0] == 0.0)
    # the error against the FP64 operator, stated
    exact = pr.ax_local(u)
    rel = float(np.max(np.abs(w - exact)) / np.max(np.abs(exact)))
    print(f"[lowp] {prec} mfma={mfma} N={N}: max|A_lo u - A u| / max|A u| = {rel:.3e}")
    assert rel < (1e-5 if prec == "f32" else 5e-2)


@pytest.mark.parametrize("mfma", [False, True], ids=["valu", "mfma"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("mesh,N", [((3, 3, 3), 5), ((4, 3, 2), 7), ((2, 2, 3), 11)])
def test_mixed_cg_small(prec, mesh, N, mfma):
    nx, ny, nz = mesh
    pr = op.Problem(nx, ny, nz, N, 0.05)
    b = workload.continuous_rhs(40 + N, nx, ny, nz, N)
    xr, _ = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, rtol=1e-12)
    A = sem.SemOperator(nx, ny, nz, N, 0.05, lowprec=prec, device=DEV, mfma=mfma)
    bg = torch.from_numpy(b).to(DEV)
    x, res = A.cg(bg, rtol=1e-8, mixed=True, inner_rtol=1e-3)
    assert res.status == 0 and res.rel_res <= 1e-8 and res.outer_iters >= 2
    xv = x.cpu().numpy()
    c = pr.c.reshape(-1)
    err = math.sqrt(np.sum(c * (xv - xr.reshape(-1)) ** 2) / np.sum(c * xr.reshape(-1) ** 2))
    print(f"[mixed] {prec} {mesh} N={N}: outer {res.outer_iters}, inner {res.iters}, "
          f"rel res {res.rel_res:.2e}, ||x-x64||/||x64|| = {err:.2e}")
    assert err <= 1e-5
    # the FP64 solve of the same system for comparison of iteration counts
    A64 = sem.SemOperator(nx, ny, nz, N, 0.05, device=DEV)
    _, r64 = A64.cg(bg, rtol=1e-8)
    print(f"[mixed] FP64 iterations {r64.iters}")


@pytest.mark.parametrize("N", list(range(1, 13)))
def test_mixed_cg_all_orders(N):
    """FP32 inner-outer CG at every order (the FP32 CG update at each order's
    tile shape) on meshes with partial update tiles."""
    mesh = (5, 3, 2) if N <= 7 else (3, 2, 3)
    pr = op.Problem(*mesh, N, 0.05)
    b = workload.continuous_rhs(80 + N, *mesh, N)
    xr, _ = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, rtol=1e-12)
    A = sem.SemOperator(*mesh, N, 0.05, lowprec="f32", device=DEV)
    x, res = A.cg(torch.from_numpy(b).to(DEV), rtol=1e-8, mixed=True)
    assert res.status == 0 and res.rel_res <= 1e-8
    xv = x.cpu().numpy()
    c = pr.c.reshape(-1)
    err = math.sqrt(np.sum(c * (xv - xr.reshape(-1)) ** 2) / np.sum(c * xr.reshape(-1) ** 2))
    assert err <= 1e-5
    assert opcg.true_rel_residual(pr.ax, pr.shape4(b), pr.shape4(xv), pr.c) <= 1e-8 * (1 + 1e-3)


@pytest.mark.parametrize("mesh", [(1, 2, 2), (2, 1, 1), (1, 1, 1)])
def test_mixed_cg_linear_update_slab_meshes(mesh):
    """FP32 inner-outer CG at N = 11, whose FP32 update is the linear tile,
    on meshes one element across and on a single element."""
    N = 11
    pr = op.Problem(*mesh, N, 0.05)
    b = workload.continuous_rhs(95, *mesh, N)
    xr, _ = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, rtol=1e-12)
    A = sem.SemOperator(*mesh, N, 0.05, lowprec="f32", device=DEV)
    x, res = A.cg(torch.from_numpy(b).to(DEV), rtol=1e-8, mixed=True)
    assert res.status == 0 and res.rel_res <= 1e-8
    xv = x.cpu().numpy()
    c = pr.c.reshape(-1)
    err = math.sqrt(np.sum(c * (xv - xr.reshape(-1)) ** 2) / np.sum(c * xr.reshape(-1) ** 2))
    assert err <= 1e-5
    assert opcg.true_rel_residual(pr.ax, pr.shape4(b), pr.shape4(xv), pr.c) <= 1e-8 * (1 + 1e-3)


def test_mixed_cg_repeatable_and_graph_stream():
    nx, ny, nz, N = 4, 4, 4, 7
    A = sem.SemOperator(nx, ny, nz, N, 0.05, lowprec="f32", device=DEV)
    bg = torch.from_numpy(workload.continuous_rhs(2, nx, ny, nz, N)).to(DEV)
    x1, r1 = A.cg(bg, rtol=1e-8, mixed=True)
    side = torch.cuda.Stream(device=DEV)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        x2, r2 = A.cg(bg, rtol=1e-8, mixed=True, check_every=10)
        x3, r3 = A.cg(bg, rtol=1e-8, mixed=True, check_every=10)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2) and torch.equal(x2, x3)
    assert r1.iters == r2.iters == r3.iters and r1.rel_res == r3.rel_res


def test_mixed_requires_lowprec_copy():
    A = sem.SemOperator(2, 2, 2, 3, 0.0, device=DEV)
    bg = torch.from_numpy(workload.continuous_rhs(2, 2, 2, 2, 3)).to(DEV)
    with pytest.raises(sem.SemError):
        A.cg(bg, rtol=1e-8, mixed=True)
    with pytest.raises(sem.SemError):
        A.ax_lowp(torch.zeros(A.L, dtype=torch.float32, device=DEV))


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mfma_operator_full_size_sampled(prec):
    """32x32x32 deformed N = 7 with the contractions on the matrix cores: on a
    sample of elements, the local result is inside the componentwise bound of
    the rounded operator evaluated by the oracle on a 27-element patch."""
    nx = ny = nz = 32
    N, amp = 7, 0.05
    A = sem.SemOperator(nx, ny, nz, N, amp, lowprec=prec, device=DEV, mfma=True)
    u = workload.iid_lvector(77, A.L).astype(np.float32)
    w = A.ax_lowp(torch.from_numpy(u).to(DEV), sem.LOCAL).cpu().numpy().astype(np.float64)
    n3 = (N + 1) ** 3
    rng = np.random.default_rng(5)
    for e in [int(v) for v in rng.integers(0, A.E, size=6)] + [0, A.E - 1]:
        pe = op.Patch(nx, ny, nz, N, amp, e)
        els = np.asarray(pe.elements)
        ue = u.astype(np.float64)[els[:, None] * n3 + np.arange(n3)].reshape(-1)
        local = types.SimpleNamespace(D=pe.D, G=pe.G, shape4=lambda v: v.reshape(-1, N + 1, N + 1, N + 1))
        ref = ax_local_rounded(local, ue, prec).reshape(len(els), -1)[pe.center_slot]
        B = ax_local_abs_bound(local, ue, prec).reshape(len(els), -1)[pe.center_slot]
        got = w[e * n3:(e + 1) * n3]
        assert np.all(np.abs(got - ref) <= _tol(prec, N) * B + 1e-30), e


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_cg_full_size(prec):
    """32x32x32 deformed N = 7: the mixed solve reaches 1e-8 in FP64 true
    residual; its distance to the FP64 solve's x is stated."""
    nx = ny = nz = 32
    N, amp = 7, 0.05
    A = sem.SemOperator(nx, ny, nz, N, amp, lowprec=prec, device=DEV)
    b = torch.from_numpy(workload.continuous_rhs(4, nx, ny, nz, N)).to(DEV)
    x, res = A.cg(b, rtol=1e-8, mixed=True)
    assert res.status == 0 and res.rel_res <= 1e-8
    x64, r64 = A.cg(b, rtol=1e-8)
    c = A.export(L.SEM_FIELD_C)
    err = math.sqrt(float((c * (x - x64) ** 2).sum()) / float((c * x64 ** 2).sum()))
    print(f"[mixed-full] {prec}: outer {res.outer_iters}, inner {res.iters}, FP64 iters {r64.iters}, "
          f"||x - x64||_c/||x64||_c = {err:.2e}")
    assert err <= 1e-5
