"""GPU parity of the generic gather-scatter (sem_gs, the compressed-row gs of
paper Sec. V-B) against the oracle's row loop on the same seeded inputs.

The kernel adds each row's copies in row order starting from 0, as the oracle
does, so every comparison is bitwise."""

import numpy as np
import pytest
import torch

import workload
from oracle import gs as ogs, mesh, operator as op

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2606_12650_amd as sem

DEV = "cuda:0"


def _run(gid, v):
    off, ids = sem.gs_csr_build(gid)
    w = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(DEV)
    sem.gs(off.to(DEV), ids.to(DEV), w)
    torch.cuda.synchronize()
    return w.cpu().numpy(), off.numpy(), ids.numpy()


@pytest.mark.parametrize("case,seed", [("random", 0), ("random_dense", 1), ("periodic", 2),
                                       ("periodic_xy", 3), ("long_rows", 4)])
def test_gs_bitwise_vs_oracle(case, seed):
    rng = np.random.default_rng(seed)
    if case == "random":
        gid = rng.integers(0, 3000, 10007)  # ragged: not a multiple of the work-group
    elif case == "random_dense":
        gid = rng.integers(0, 40, 5000)  # rows of ~125 copies: the looped path
    elif case == "periodic":
        gid = ogs.periodic_global_ids(3, 2, 4, 5)
    elif case == "periodic_xy":
        gid = ogs.periodic_global_ids(4, 3, 2, 7, periodic=(True, True, False))
    else:
        gid = np.concatenate([np.full(37, 5), rng.integers(6, 900, 2000), np.full(9, 3)])
        gid = rng.permutation(gid)
    print(f"[gs] case={case} seed={seed} n={gid.size}", flush=True)
    v = workload.iid_lvector(100 + seed, gid.size)
    out, off, ids = _run(gid, v)
    ref = ogs.gs_csr(v, off, ids)
    assert np.array_equal(out, ref)
    # and the plain definition of direct stiffness summation, in ascending L order
    assert np.array_equal(out, op.dssum_fast(v, np.unique(gid, return_inverse=True)[1]))


def test_gs_no_shared_ids_and_empty():
    v = workload.iid_lvector(7, 1000)
    out, off, ids = _run(np.arange(1000)[::-1].copy(), v)
    assert off.tolist() == [0] and np.array_equal(out, v)
    w = torch.zeros(0, dtype=torch.float64, device=DEV)
    sem.gs(torch.zeros(1, dtype=torch.int32, device=DEV), torch.zeros(0, dtype=torch.int32, device=DEV), w)
    torch.cuda.synchronize()


@pytest.mark.parametrize("nx,ny,nz,N", [(3, 2, 2, 7), (2, 3, 3, 4)])
def test_gs_after_local_operator_equals_assembled(nx, ny, nz, N):
    """A_L u followed by sem_gs over the box mesh's global ids equals sem_ax's
    own fused assembly (the copies are added in another order there)."""
    A = sem.SemOperator(nx, ny, nz, N, 0.05, device=DEV)
    u = torch.from_numpy(workload.iid_lvector(21, A.L)).to(DEV)
    wl = A.ax(u, sem.LOCAL)
    wa = A.ax(u, sem.ASSEMBLED)
    off, ids = sem.gs_csr_build(mesh.global_ids(nx, ny, nz, N))
    sem.gs(off.to(DEV), ids.to(DEV), wl)
    torch.cuda.synchronize()
    a, b = wl.cpu().numpy(), wa.cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))
    A.close()


def test_gs_full_size_box_bitwise():
    """The 32x32x32, N = 7 box (16.8 M entries, 4.5 M rows) in the launch the
    bench times, bitwise against the definition (sums in ascending L order)."""
    gid = mesh.global_ids(32, 32, 32, 7)
    v = workload.iid_lvector(4, gid.size)
    print(f"[gs] full size n={gid.size}", flush=True)
    out, off, ids = _run(gid, v)
    assert off.size - 1 == int((np.bincount(gid) >= 2).sum())
    assert np.array_equal(out, op.dssum_fast(v, gid))


@pytest.mark.parametrize("amp", [0.0, 0.05])
def test_periodic_operator_from_local_operator_and_gs(amp):
    """A mesh the box index arithmetic cannot assemble: the fully periodic box
    (the deformation vanishes on the box faces, so the geometry is periodic
    too).  sem_ax(LOCAL) followed by sem_gs over the periodic ids against the
    oracle's element operator and row loop, and the symmetry of the result in
    the multiplicity-weighted inner product for continuous periodic u, v."""
    nx, ny, nz, N = 3, 2, 4, 5
    gid = ogs.periodic_global_ids(nx, ny, nz, N)
    pr = op.Problem(nx, ny, nz, N, amp)
    A = sem.SemOperator(nx, ny, nz, N, amp, device=DEV)
    off, ids = sem.gs_csr_build(gid)
    off_d, ids_d = off.to(DEV), ids.to(DEV)
    rng = np.random.default_rng(31)
    nu = int(gid.max()) + 1
    u, v = rng.uniform(-1, 1, nu)[gid], rng.uniform(-1, 1, nu)[gid]
    outs = []
    for x in (u, v):
        w = A.ax(torch.from_numpy(x).to(DEV), sem.LOCAL)
        sem.gs(off_d, ids_d, w)
        torch.cuda.synchronize()
        outs.append(w.cpu().numpy())
    ref_u = ogs.gs_csr(pr.ax_local(u).reshape(-1), off.numpy(), ids.numpy())
    assert np.max(np.abs(outs[0] - ref_u)) <= 1e-12 * np.max(np.abs(ref_u))
    c = 1.0 / op.multiplicity(gid)
    a, b = np.sum(c * u * outs[1]), np.sum(c * v * outs[0])
    assert abs(a - b) <= 1e-12 * np.sum(np.abs(c * u * outs[1]))
    # constants are in the null space of the periodic operator
    w1 = A.ax(torch.ones(A.L, dtype=torch.float64, device=DEV), sem.LOCAL)
    sem.gs(off_d, ids_d, w1)
    torch.cuda.synchronize()
    assert np.max(np.abs(w1.cpu().numpy())) <= 1e-12 * np.max(np.abs(outs[0]))
    A.close()
