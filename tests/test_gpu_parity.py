"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (written here, derived in the design notes):
  A.u (FP64)            max|w_gpu - w_ref| <= 1e-12 * max|w_ref|
  setup fields          max|f_gpu - f_ref| <= 1e-13 * max|f_ref| (G, Minv)
  dots                  |dot_gpu - dot_exact| <= 1e-13 * sum|x_i y_i w_i|
  axpy                  |y_gpu - y_ref| <= 2^-52 * (|y| + |alpha x|) elementwise
  CG, fixed iterations  ||x_gpu - x_ref||_c / ||x_ref||_c <= 1e-9
  CG, tolerance mode    both true residuals <= rtol (1 + 1e-3); iterations within 2
"""

import ctypes
import math
import os

import numpy as np
import pytest
import torch

import workload
from oracle import operator as op, pcg as opcg
from oracle.dots import abs_sum, dot_exact

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2606_12650_amd as sem
    from paper_2606_12650_amd import _lib as L

DEV = "cuda:0"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to(DEV)


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel_inf(a, ref):
    return float(np.max(np.abs(a - ref)) / max(np.max(np.abs(ref)), 1e-300))


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"[gpu-test] {os.environ.get('PYTEST_CURRENT_TEST', '')}", flush=True)


# ------------------------------------------------------------------ setup (a1)

@pytest.mark.parametrize("N", list(range(1, 13)))
def test_setup_fields_match_oracle(N):
    nx, ny, nz, amp = 3, 2, 2, 0.05
    pr = op.Problem(nx, ny, nz, N, amp)
    A = sem.SemOperator(nx, ny, nz, N, amp, device=DEV)
    nodes = _cpu(A.export(L.SEM_FIELD_NODES))
    assert np.max(np.abs(nodes[:N + 1] - pr.xi)) <= 4e-16
    assert np.max(np.abs(nodes[N + 1:] - pr.w) / pr.w) <= 1e-14
    D = _cpu(A.export(L.SEM_FIELD_D)).reshape(N + 1, N + 1)
    assert _rel_inf(D, pr.D) <= 1e-13
    G = _cpu(A.export(L.SEM_FIELD_G)).reshape(pr.G.shape)
    assert _rel_inf(G, pr.G) <= 1e-13
    minv = _cpu(A.export(L.SEM_FIELD_MINV)).reshape(pr.minv.shape)
    assert _rel_inf(minv, pr.minv) <= 1e-13
    assert np.all(minv[pr.mask == 0] == 0.0)
    c = _cpu(A.export(L.SEM_FIELD_C)).reshape(pr.c.shape)
    assert np.array_equal(c, pr.c)


# ------------------------------------------------------------------ A.u (a2-a5)

MFMA = pytest.mark.parametrize("mfma", [False, True], ids=["valu", "mfma"])


def _same_on_copies(pr, v):
    gid = pr.gid.reshape(-1)
    hi = np.full(gid.max() + 1, -np.inf)
    lo = np.full(gid.max() + 1, np.inf)
    np.maximum.at(hi, gid, v.reshape(-1))
    np.minimum.at(lo, gid, v.reshape(-1))
    return bool(np.array_equal(hi, lo))


@MFMA
@pytest.mark.parametrize("N", list(range(1, 13)))
@pytest.mark.parametrize("amp", [0.0, 0.05])
def test_ax_all_orders(N, amp, mfma):
    nx, ny, nz = 3, 2, 2
    pr = op.Problem(nx, ny, nz, N, amp)
    A = sem.SemOperator(nx, ny, nz, N, amp, device=DEV, mfma=mfma)
    u_disc = workload.iid_lvector(100 + N, pr.L)
    u_cont = workload.continuous_rhs(200 + N, nx, ny, nz, N, zero_boundary=False)
    w = _cpu(A.ax(_gpu(u_disc), sem.LOCAL)).reshape(pr.mask.shape)
    assert _rel_inf(w, pr.ax_local(u_disc)) <= 1e-12
    w = _cpu(A.ax(_gpu(u_cont), sem.ASSEMBLED)).reshape(pr.mask.shape)
    assert _rel_inf(w, pr.ax_assembled(u_cont)) <= 1e-12
    ref = pr.ax(u_cont)
    w = _cpu(A.ax(_gpu(u_cont), sem.MASKED)).reshape(pr.mask.shape)
    assert _rel_inf(w, ref) <= 1e-12
    assert np.all(w[pr.mask == 0] == 0.0)
    # the assembled result holds the same bits on every copy of a node
    wa = _cpu(A.ax(_gpu(u_disc), sem.ASSEMBLED))
    assert _same_on_copies(pr, wa)


@pytest.mark.parametrize("mesh,N", [((1, 1, 1), 1), ((1, 1, 1), 7), ((1, 1, 1), 12),
                                    ((5, 1, 1), 3), ((1, 7, 1), 5), ((3, 3, 5), 7),
                                    ((2, 3, 4), 11), ((7, 5, 3), 2)])
@MFMA
def test_ax_ragged_and_degenerate_meshes(mesh, N, mfma):
    """Element counts that leave the last work-group partly empty, single
    elements (every node on the boundary) and slab meshes."""
    nx, ny, nz = mesh
    pr = op.Problem(nx, ny, nz, N, 0.05)
    A = sem.SemOperator(nx, ny, nz, N, 0.05, device=DEV, mfma=mfma)
    u = workload.iid_lvector(7, pr.L)
    for mode, ref in ((sem.LOCAL, pr.ax_local(u)), (sem.ASSEMBLED, pr.ax_assembled(u)),
                      (sem.MASKED, pr.ax(u))):
        w = _cpu(A.ax(_gpu(u), mode)).reshape(pr.mask.shape)
        assert _rel_inf(w, ref) <= 1e-12, mode


def test_ax_config1_and_repeatability():
    """4x4x4 affine elements at N=7 (32768 L-entries)."""
    nx = ny = nz = 4
    N = 7
    pr = op.Problem(nx, ny, nz, N, 0.0)
    A = sem.SemOperator(nx, ny, nz, N, 0.0, device=DEV)
    u = workload.continuous_rhs(1, nx, ny, nz, N)
    ug = _gpu(u)
    w1 = A.ax(ug)
    w2 = A.ax(ug)
    assert torch.equal(w1, w2)
    assert _rel_inf(_cpu(w1).reshape(pr.mask.shape), pr.ax(u)) <= 1e-12
    # A annihilates constants before assembly and masking
    one = torch.ones(pr.L, dtype=torch.float64, device=DEV)
    wl = _cpu(A.ax(one, sem.LOCAL))
    assert np.max(np.abs(wl)) <= 1e-12 * np.max(np.abs(pr.ax_local(u)))


@MFMA
def test_ax_full_size_sampled(mfma):
    """The 32x32x32 deformed N=7 mesh (16.8 M L-entries) in the launch shape
    the bench times; the oracle evaluates sampled elements from their
    neighbourhoods."""
    nx = ny = nz = 32
    N, amp = 7, 0.05
    A = sem.SemOperator(nx, ny, nz, N, amp, device=DEV, mfma=mfma)
    u = workload.continuous_rhs(4, nx, ny, nz, N)
    ug = _gpu(u)
    n3 = (N + 1) ** 3
    wm = _cpu(A.ax(ug, sem.MASKED))
    wl = _cpu(A.ax(ug, sem.LOCAL))
    rng = np.random.default_rng(0)
    centers = [0, nx * ny * nz - 1, 31, 32 * 32 * 16 + 32 * 16 + 16] + list(rng.integers(0, nx * ny * nz, 6))
    for c in centers:
        P = op.Patch(nx, ny, nz, N, amp, int(c))
        up = np.concatenate([u[e * n3:(e + 1) * n3] for e in P.elements])
        ref = P.ax_center(up, "masked").reshape(-1)
        got = wm[c * n3:(c + 1) * n3]
        scale = max(np.max(np.abs(ref)), 1e-300)
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale, c
        refl = P.ax_center(up, "local").reshape(-1)
        assert np.max(np.abs(wl[c * n3:(c + 1) * n3] - refl)) <= 1e-12 * np.max(np.abs(refl)), c


# ------------------------------------------------------------------ vectors (a6, a7)

@pytest.mark.parametrize("n", [0, 1, 7, 2047, 2048, 2049, 32768, 1000003])
def test_axpy_and_dot(n):
    x = workload.iid_lvector(31, n)
    y = workload.iid_lvector(32, n)
    c = np.random.default_rng(33).choice([1.0, 0.5, 0.25, 0.125], n)
    xg, yg, cg = _gpu(x), _gpu(y), _gpu(c)
    d = _cpu(sem.vec_dot(xg, yg))[0]
    assert abs(d - dot_exact(x, y)) <= 1e-13 * abs_sum(x, y) + 1e-300
    dw = _cpu(sem.vec_dot(xg, yg, cg))[0]
    assert abs(dw - dot_exact(x, y, c)) <= 1e-13 * abs_sum(x, y, c) + 1e-300
    assert _cpu(sem.vec_dot(xg, yg))[0] == d  # bitwise repeatable
    alpha = 0.5
    yy = yg.clone()
    sem.vec_axpy(alpha, xg, yy)
    got = _cpu(yy)
    ref = alpha * x + y
    assert np.all(np.abs(got - ref) <= 2.0 ** -52 * (np.abs(y) + np.abs(alpha * x)))


def test_dot_norm_relative():
    """A norm (no cancellation) within 1e-13 of its exact value."""
    x = workload.iid_lvector(41, 3 * 10 ** 5)
    d = _cpu(sem.vec_dot(_gpu(x), _gpu(x)))[0]
    assert abs(d - dot_exact(x, x)) <= 1e-13 * dot_exact(x, x)


# ------------------------------------------------------------------ CG (a8)

def _c_norm(v, c):
    return math.sqrt(float(np.sum(c.reshape(-1) * v.reshape(-1) ** 2)))


@MFMA
def test_cg_fixed_iterations_config1(mfma):
    """4x4x4 affine, N=7, 50 Jacobi-PCG iterations from x = 0."""
    nx = ny = nz = 4
    N = 7
    pr = op.Problem(nx, ny, nz, N, 0.0)
    b = workload.continuous_rhs(2, nx, ny, nz, N)
    xr, info = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, fixed_iter=50, history=True)
    A = sem.SemOperator(nx, ny, nz, N, 0.0, device=DEV, mfma=mfma)
    xg, res = A.cg(_gpu(b), fixed_iter=50)
    assert res.iters == 50 and res.status == 0
    x = _cpu(xg)
    err = _c_norm(x - xr.reshape(-1), pr.c) / _c_norm(xr, pr.c)
    assert err <= 1e-9
    assert abs(res.rel_res - info["rel_res"]) <= 1e-6 * info["rel_res"]
    # the recursive residual history of the first 20 iterations
    xh = torch.empty_like(xg)
    for k in range(1, 21):
        _, rk = A.cg(_gpu(b), xh, fixed_iter=k)
        ref = info["res_hist"][k - 1]
        assert abs(rk.rel_res - ref) <= 1e-6 * ref, (k, rk.rel_res, ref)
    # a second solve gives the same bits (fixed reduction order), also when it
    # runs as a captured graph on a side stream
    x2, res2 = A.cg(_gpu(b), fixed_iter=50)
    assert torch.equal(xg, x2) and res2.rel_res == res.rel_res
    side = torch.cuda.Stream(device=DEV)
    bg = _gpu(b)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for every in (50, 10, 10):
            x3, res3 = A.cg(bg, fixed_iter=50, check_every=every)
            assert res3.iters == 50
    torch.cuda.synchronize()
    assert torch.equal(xg, x3) and res3.rel_res == res.rel_res


@pytest.mark.parametrize("mesh,N,every", [((5, 4, 3), 7, 25), ((3, 3, 3), 5, 7), ((4, 3, 2), 9, 1),
                                          ((2, 3, 2), 11, 10)])
@MFMA
def test_cg_tolerance_mode(mesh, N, every, mfma):
    nx, ny, nz = mesh
    pr = op.Problem(nx, ny, nz, N, 0.05)
    b = workload.continuous_rhs(4, nx, ny, nz, N)
    xr, info = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, rtol=1e-8)
    A = sem.SemOperator(nx, ny, nz, N, 0.05, device=DEV, mfma=mfma)
    xg, res = A.cg(_gpu(b), rtol=1e-8, check_every=every)
    assert res.status == 0 and res.rel_res <= 1e-8
    assert abs(res.iters - info["iters"]) <= 2
    x = _cpu(xg)
    tr_gpu = opcg.true_rel_residual(pr.ax, pr.shape4(b), pr.shape4(x), pr.c)
    tr_ref = opcg.true_rel_residual(pr.ax, pr.shape4(b), xr, pr.c)
    assert tr_gpu <= 1e-8 * (1 + 1e-3) and tr_ref <= 1e-8 * (1 + 1e-3)
    assert _c_norm(x - xr.reshape(-1), pr.c) / _c_norm(xr, pr.c) <= 1e-5


@pytest.mark.parametrize("N", list(range(1, 13)))
def test_cg_all_orders_ragged(N):
    """20 FP64 PCG iterations at every order on meshes whose element count and
    x extent are not multiples of the update tiles' element groups (partial
    last tiles, tiles that straddle element rows)."""
    mesh = (5, 3, 2) if N <= 7 else (3, 2, 3)
    pr = op.Problem(*mesh, N, 0.05)
    b = workload.continuous_rhs(60 + N, *mesh, N)
    xr, info = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, fixed_iter=20)
    A = sem.SemOperator(*mesh, N, 0.05, device=DEV)
    xg, res = A.cg(_gpu(b), fixed_iter=20)
    assert res.iters == 20 and res.status == 0
    x = _cpu(xg)
    assert _c_norm(x - xr.reshape(-1), pr.c) / _c_norm(xr, pr.c) <= 1e-9
    # small systems converge exactly within 20 iterations: past that the
    # residuals are rounding noise on both sides
    assert (abs(res.rel_res - info["rel_res"]) <= 1e-6 * info["rel_res"]
            or max(res.rel_res, info["rel_res"]) <= 1e-13)
    # continuity: every copy of a node holds the same bits of x
    assert _same_on_copies(pr, x)


@pytest.mark.parametrize("mesh,N", [((1, 3, 2), 9), ((2, 1, 3), 10), ((3, 2, 1), 11), ((1, 1, 1), 11),
                                    ((1, 1, 4), 9), ((4, 1, 1), 10)])
def test_cg_linear_update_slab_meshes(mesh, N):
    """20 FP64 PCG iterations at orders whose update runs the linear tile, on
    meshes one element across in some direction and on a single element: a
    thread's items there step over element rows, columns and layers at once."""
    pr = op.Problem(*mesh, N, 0.05)
    b = workload.continuous_rhs(90 + N, *mesh, N)
    xr, info = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, fixed_iter=20)
    A = sem.SemOperator(*mesh, N, 0.05, device=DEV)
    xg, res = A.cg(_gpu(b), fixed_iter=20)
    assert res.iters == 20 and res.status == 0
    x = _cpu(xg)
    assert _c_norm(x - xr.reshape(-1), pr.c) / _c_norm(xr, pr.c) <= 1e-9
    assert (abs(res.rel_res - info["rel_res"]) <= 1e-6 * info["rel_res"]
            or max(res.rel_res, info["rel_res"]) <= 1e-13)
    assert _same_on_copies(pr, x)


@pytest.mark.parametrize("mesh,N", [((5, 3, 2), 3), ((3, 3, 2), 7), ((3, 2, 3), 9), ((2, 3, 2), 11)])
@MFMA
def test_plain_cg_matches_oracle(mesh, N, mfma):
    """The unpreconditioned CG (SEM_PRECOND_NONE, the paper's Nekbone CG)
    against the oracle's CG with Minv = mask: 20 fixed iterations, then
    tolerance mode; the same context then runs Jacobi-PCG again and must give
    the bits of a Jacobi-PCG run that never saw the plain mode (the captured
    iteration graph is keyed by the preconditioner)."""
    pr = op.Problem(*mesh, N, 0.05)
    b = workload.continuous_rhs(80 + N, *mesh, N)
    A = sem.SemOperator(*mesh, N, 0.05, device=DEV, mfma=mfma)
    xr, info = opcg.pcg(pr.ax, pr.shape4(b), pr.mask, pr.c, fixed_iter=20)
    xg, res = A.cg(_gpu(b), fixed_iter=20, precond=False)
    assert res.iters == 20 and res.status == 0
    x = _cpu(xg)
    assert _c_norm(x - xr.reshape(-1), pr.c) / _c_norm(xr, pr.c) <= 1e-9
    assert abs(res.rel_res - info["rel_res"]) <= 1e-6 * info["rel_res"]
    assert _same_on_copies(pr, x)
    xr, info = opcg.pcg(pr.ax, pr.shape4(b), pr.mask, pr.c, rtol=1e-8)
    xg, res = A.cg(_gpu(b), rtol=1e-8, precond=False)
    assert res.status == 0 and abs(res.iters - info["iters"]) <= 2
    tr = opcg.true_rel_residual(pr.ax, pr.shape4(b), pr.shape4(_cpu(xg)), pr.c)
    assert tr <= 1e-8 * (1 + 1e-3)
    xj, resj = A.cg(_gpu(b), rtol=1e-8)
    B = sem.SemOperator(*mesh, N, 0.05, device=DEV, mfma=mfma)
    xj2, resj2 = B.cg(_gpu(b), rtol=1e-8)
    assert torch.equal(xj, xj2) and resj.iters == resj2.iters


def test_precond_option_is_checked():
    A = sem.SemOperator(2, 2, 2, 3, 0.0, lowprec="f32", device=DEV)
    b = _gpu(workload.continuous_rhs(1, 2, 2, 2, 3))
    lib = L.lib()
    x = torch.empty_like(b)
    info = L.SemCgInfo()
    for precond, mixed in ((2, 0), (-1, 0), (L.SEM_PRECOND_NONE, 1)):
        opts = L.SemCgOpts(1e-8, 0, 0, mixed, 0, 0.0, 0, precond)
        rc = lib.sem_cg(A._ctx, sem.sem._ptr(b), sem.sem._ptr(x), ctypes.byref(opts), ctypes.byref(info),
                        sem.sem._stream(A.device))
        assert rc == L.SEM_ERR_ARG


def test_cg_breakdown_and_cap_are_reported():
    nx = ny = nz = 2
    N = 4
    A = sem.SemOperator(nx, ny, nz, N, 0.05, device=DEV)
    b = workload.continuous_rhs(5, nx, ny, nz, N)
    bn = b.copy()
    bn[np.flatnonzero(b)[0]] = np.nan
    _, res = A.cg(_gpu(bn), rtol=1e-8, raise_on_fail=False)
    assert res.status == L.SEM_ERR_BREAKDOWN
    _, res = A.cg(_gpu(b), rtol=1e-14, max_iter=3, raise_on_fail=False)
    assert res.status == L.SEM_ERR_NOTCONV and res.iters == 3
    # the operator still works after failed solves
    _, res = A.cg(_gpu(b), rtol=1e-8)
    assert res.status == 0
    zero = torch.zeros(A.L, dtype=torch.float64, device=DEV)
    x, res = A.cg(zero, rtol=1e-8)
    assert res.status == 0 and res.iters == 0 and float(x.abs().max()) == 0.0


def test_cg_full_size_properties():
    """32x32x32 deformed N=7 to 1e-8: properties that hold at any size (the
    oracle's full-size solve is too slow for a test): convergence, a true
    residual consistent with the recursive one, bitwise repeatability."""
    nx = ny = nz = 32
    N, amp = 7, 0.05
    A = sem.SemOperator(nx, ny, nz, N, amp, device=DEV)
    b = _gpu(workload.continuous_rhs(4, nx, ny, nz, N))
    x, res = A.cg(b, rtol=1e-8)
    assert res.status == 0 and res.rel_res <= 1e-8 and 50 < res.iters < 5000
    r = b - A.ax(x)
    c = A.export(L.SEM_FIELD_C)
    bm = b * (A.export(L.SEM_FIELD_MINV) != 0)
    tr = math.sqrt(float((c * r * r).sum()) / float((c * bm * bm).sum()))
    assert tr <= 1e-8 * (1 + 1e-3)
    x2, res2 = A.cg(b, rtol=1e-8)
    assert torch.equal(x, x2) and res2.iters == res.iters
