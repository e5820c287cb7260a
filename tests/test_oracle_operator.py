"""Pins of the oracle's mesh, geometric factors, element operator, dssum,
mask, Jacobi diagonal and CG.

The checks come from outside the oracle: the Kronecker-sum closed form of an
affine element, a dense brute-force assembly from a Legendre-Vandermonde
basis, null space, symmetry and positivity, exact node counts, a dense direct
solve, and spectral convergence to a manufactured solution.  The last tests
plant plausible mistakes in copies of the oracle's routines and check that
the pins above reject them.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

import workload
from oracle import brute, operator as op, pcg as opcg
from oracle.dots import dot_exact
from oracle.mesh import n_unique


def _problem(nx, ny, nz, N, amp, fast=True):
    return op.Problem(nx, ny, nz, N, amp, fast_dssum=fast)


def _kron_element(N, h):
    """(h/2) (K x M x M + M x K x M + M x M x K) on a cube of side h,
    K = 1-D reference stiffness, M = diag(w)."""
    from oracle.gll import deriv_matrix, gll_nodes_weights
    _, w = gll_nodes_weights(N)
    D = deriv_matrix(N)
    K = D.T @ np.diag(w) @ D
    M = sp.diags(w)
    K = sp.csr_matrix(K)
    A = sp.kron(sp.kron(M, M), K) + sp.kron(sp.kron(M, K), M) + sp.kron(sp.kron(K, M), M)
    return (h / 2.0) * A.toarray()


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_affine_element_is_kronecker_sum(N):
    pr = _problem(1, 1, 1, N, 0.0)
    n3 = (N + 1) ** 3
    A = np.zeros((n3, n3))
    for col in range(n3):
        e = np.zeros(n3)
        e[col] = 1.0
        A[:, col] = pr.ax_local(e).reshape(-1)
    ref = _kron_element(N, 1.0)
    assert np.max(np.abs(A - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_worked_value_trilinear_unit_cube():
    """N = 1 on [0,1]^3: diagonal 3/4, edge neighbours -1/4, all others 0."""
    pr = _problem(1, 1, 1, 1, 0.0)
    A = np.stack([pr.ax_local(np.eye(8)[c]).reshape(-1) for c in range(8)], axis=1)
    for a in range(8):
        for b in range(8):
            ham = bin(a ^ b).count("1")
            expect = 0.75 if ham == 0 else (-0.25 if ham == 1 else 0.0)
            assert abs(A[a, b] - expect) < 1e-15


@pytest.mark.parametrize("N,amp", [(3, 0.0), (5, 0.05), (7, 0.05)])
def test_constants_in_null_space(N, amp):
    pr = _problem(2, 2, 2, N, amp)
    one = np.ones(pr.L)
    out = pr.ax_local(one)
    scale = np.max(np.abs(pr.G)) * np.max(np.abs(pr.D)) ** 2 * (N + 1) ** 2
    assert np.max(np.abs(out)) <= 1e-13 * scale


@pytest.mark.parametrize("N,amp", [(4, 0.05), (7, 0.05)])
def test_symmetry(N, amp):
    pr = _problem(2, 2, 2, N, amp)
    u = workload.iid_lvector(11, pr.L)
    v = workload.iid_lvector(12, pr.L)
    Au = pr.ax_local(u).reshape(-1)
    Av = pr.ax_local(v).reshape(-1)
    lhs, rhs = dot_exact(v, Au), dot_exact(u, Av)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(v * Au))
    # assembled, masked, continuous vectors with the c-weighted inner product
    uc = workload.continuous_rhs(13, 2, 2, 2, N)
    vc = workload.continuous_rhs(14, 2, 2, 2, N)
    Auc = pr.ax(uc).reshape(-1)
    Avc = pr.ax(vc).reshape(-1)
    c = pr.c.reshape(-1)
    lhs, rhs = dot_exact(vc, Auc, c), dot_exact(uc, Avc, c)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(c * vc * Auc))


@pytest.mark.parametrize("N,amp", [(3, 0.0), (6, 0.05), (9, 0.05)])
def test_geometry_valid_and_volume(N, amp):
    pr = _problem(2, 3, 2, N, amp)
    assert np.all(pr.detJ > 0)
    wq = np.einsum("k,j,i->kji", pr.w, pr.w, pr.w)
    vol = np.sum(wq[None] * pr.detJ)
    # The map adds one scalar f to all three coordinates, so det J = h^3/8 *
    # (1 + (2/h)(f_r + f_s + f_t)) (a rank-one update); GLL quadrature is exact
    # on it and the f terms telescope to the box boundary, where the
    # interpolated f is 0: the volume is 1 to rounding, deformed or not.
    assert abs(vol - 1.0) < 1e-13
    G = pr.G
    M = np.stack([np.stack([G[:, 0], G[:, 1], G[:, 2]], -1),
                  np.stack([G[:, 1], G[:, 3], G[:, 4]], -1),
                  np.stack([G[:, 2], G[:, 4], G[:, 5]], -1)], -1)
    assert np.all(np.linalg.eigvalsh(M) > 0)


@pytest.mark.parametrize("mesh,N,amp", [((1, 1, 1), 3, 0.0), ((2, 2, 2), 2, 0.05),
                                        ((2, 3, 2), 3, 0.05), ((3, 3, 3), 2, 0.05),
                                        ((2, 2, 2), 4, 0.05)])
def test_brute_force_dense_matches(mesh, N, amp):
    nx, ny, nz = mesh
    pr = _problem(nx, ny, nz, N, amp, fast=False)
    K = brute.element_matrices(pr.coords, pr.xi, pr.w, N)
    ng = n_unique(nx, ny, nz, N)
    A = brute.assemble_dense(K, pr.gid, ng)
    assert np.max(np.abs(A - A.T)) <= 1e-13 * np.max(np.abs(A))
    lattice = workload.random_lattice(21, nx, ny, nz, N, zero_boundary=False)
    ubar = lattice.reshape(-1)
    u = workload.lattice_to_lvector(lattice, nx, ny, nz, N).reshape(-1)
    Au = pr.ax(u).reshape(-1)
    ref = (A @ ubar)[pr.gid]
    interior = pr.mask.reshape(-1) > 0
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(Au[interior] - ref[interior])) <= 1e-12 * scale
    assert np.all(Au[~interior] == 0.0)
    # Dirichlet-reduced matrix is SPD; its diagonal is the Jacobi diagonal.
    inner = np.unique(pr.gid[interior])
    Ar = A[np.ix_(inner, inner)]
    if Ar.size:
        assert np.min(np.linalg.eigvalsh(Ar)) > 0
        dg = np.zeros(ng)
        dg[pr.gid] = pr.diag.reshape(-1)
        assert np.max(np.abs(dg[inner] - np.diag(Ar))) <= 1e-13 * np.max(np.abs(np.diag(Ar)))


@pytest.mark.parametrize("nx,ny,nz,N", [(4, 4, 4, 7), (2, 3, 4, 5), (1, 1, 1, 3)])
def test_counts_and_multiplicity(nx, ny, nz, N):
    pr = _problem(nx, ny, nz, N, 0.0)
    assert pr.L == nx * ny * nz * (N + 1) ** 3
    assert math.isclose(pr.c.sum(), n_unique(nx, ny, nz, N), rel_tol=0, abs_tol=1e-9)
    interior = np.unique(pr.gid[pr.mask.reshape(-1) > 0]).size
    assert interior == (nx * N - 1) * (ny * N - 1) * (nz * N - 1)
    if (nx, ny, nz, N) == (4, 4, 4, 7):
        assert pr.L == 32768 and n_unique(4, 4, 4, 7) == 24389 and interior == 19683


def test_dssum_slow_equals_fast_and_idempotence():
    pr_s = _problem(2, 3, 2, 3, 0.05, fast=False)
    v = workload.iid_lvector(5, pr_s.L).reshape(pr_s.mask.shape)
    a = op.dssum(v, pr_s.gid)
    b = op.dssum_fast(v, pr_s.gid)
    assert np.array_equal(a, b)
    np.testing.assert_allclose(op.dssum(a, pr_s.gid), pr_s.mult * a, rtol=1e-15, atol=1e-14)
    # a continuous vector is unchanged by dssum up to the multiplicity
    u = workload.continuous_rhs(6, 2, 3, 2, 3, zero_boundary=False).reshape(pr_s.mask.shape)
    np.testing.assert_allclose(op.dssum(u, pr_s.gid), pr_s.mult * u, rtol=1e-15)


@pytest.mark.parametrize("mesh,N,amp", [((2, 2, 2), 3, 0.05), ((2, 3, 2), 4, 0.05)])
def test_pcg_matches_dense_solve(mesh, N, amp):
    nx, ny, nz = mesh
    pr = _problem(nx, ny, nz, N, amp)
    K = brute.element_matrices(pr.coords, pr.xi, pr.w, N)
    ng = n_unique(nx, ny, nz, N)
    A = brute.assemble_dense(K, pr.gid, ng)
    lattice = workload.random_lattice(31, nx, ny, nz, N)
    b = workload.lattice_to_lvector(lattice, nx, ny, nz, N).reshape(-1)
    inner = np.unique(pr.gid[pr.mask.reshape(-1) > 0])
    xs = np.zeros(ng)
    xs[inner] = np.linalg.solve(A[np.ix_(inner, inner)], lattice.reshape(-1)[inner])
    x, info = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, rtol=1e-12)
    assert info["converged"]
    kappa = np.linalg.cond(A[np.ix_(inner, inner)])
    err = np.max(np.abs(x.reshape(-1) - xs[pr.gid])) / np.max(np.abs(xs))
    assert err <= kappa * 1e-12


def test_pcg_fixed_iterations_and_residual_decay():
    pr = _problem(4, 4, 4, 7, 0.0)
    b = workload.continuous_rhs(2, 4, 4, 4, 7)
    x, info = opcg.pcg(pr.ax, pr.shape4(b), pr.minv, pr.c, fixed_iter=50, history=True)
    assert info["iters"] == 50
    h = info["res_hist"]
    assert h[-1] < 1e-2 * h[0]
    tr = opcg.true_rel_residual(pr.ax, pr.shape4(b), x, pr.c)
    assert abs(tr - info["rel_res"]) < 1e-6


@pytest.mark.slow
def test_manufactured_solution_converges_spectrally():
    """-Lap u = 3 pi^2 u for u = sin(pi x) sin(pi y) sin(pi z): the nodal error
    falls exponentially with N at fixed E."""
    errs = []
    for N in (2, 4, 6, 8):
        pr = _problem(2, 2, 2, N, 0.0)
        X, Y, Z = pr.coords
        us = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
        wq = np.einsum("k,j,i->kji", pr.w, pr.w, pr.w)
        bl = wq[None] * pr.detJ * 3 * np.pi ** 2 * us
        b = pr.mask * pr.dssum(bl)
        x, info = opcg.pcg(pr.ax, b, pr.minv, pr.c, rtol=1e-13)
        errs.append(np.max(np.abs(x - us)))
    assert errs[-1] < 1e-6
    for a, b in zip(errs, errs[1:]):
        assert b < a / 5


# ---------------------------------------------------------------------------
# Planted mistakes: copies of the oracle's operator with one plausible error
# each must fail the pins used above.

def _ax_mutant(kind):
    def f(u, D, G):
        ur, us, ut = op.grad_ref(D, u)
        if kind == "transposed_grad":
            ur = np.einsum("li,ekjl->ekji", D, u)
        grr, grs, grt, gss, gst, gtt = (G[:, q] for q in range(6))
        wr = grr * ur + grs * us + grt * ut
        ws = (0 if kind == "dropped_rs" else grs) * ur + gss * us + gst * ut
        wt = grt * ur + gst * us + gtt * ut
        out = np.einsum("li,ekjl->ekji", D, wr)
        out += np.einsum("lj,ekli->ekji", D, ws)
        if kind == "wrong_sign":
            out -= np.einsum("lk,elji->ekji", D, wt)
        elif kind == "transposed_div":
            out += np.einsum("kl,elji->ekji", D, wt)
        else:
            out += np.einsum("lk,elji->ekji", D, wt)
        return out
    return f


@pytest.mark.parametrize("kind", ["transposed_grad", "dropped_rs", "wrong_sign", "transposed_div"])
def test_planted_operator_mistakes_are_caught(kind):
    nx, ny, nz, N, amp = 2, 2, 2, 3, 0.05
    pr = _problem(nx, ny, nz, N, amp)
    K = brute.element_matrices(pr.coords, pr.xi, pr.w, N)
    A = brute.assemble_dense(K, pr.gid, n_unique(nx, ny, nz, N))
    lattice = workload.random_lattice(21, nx, ny, nz, N, zero_boundary=False)
    u = workload.lattice_to_lvector(lattice, nx, ny, nz, N)
    mut = _ax_mutant(kind)
    Au = (pr.mask * pr.dssum(mut(u, pr.D, pr.G))).reshape(-1)
    ref = (A @ lattice.reshape(-1))[pr.gid]
    interior = pr.mask.reshape(-1) > 0
    bad_brute = np.max(np.abs(Au[interior] - ref[interior])) > 1e-12 * np.max(np.abs(ref))
    one = np.ones_like(u)
    bad_null = np.max(np.abs(mut(one, pr.D, pr.G))) > 1e-10
    assert bad_brute or bad_null


def test_planted_geometry_mistake_is_caught():
    """A metric built from J^-T instead of J^-1 changes G on deformed
    elements; the brute-force assembly (adjugate route) rejects it."""
    nx, ny, nz, N = 2, 2, 2, 3
    pr = _problem(nx, ny, nz, N, 0.05)
    X, Y, Z = pr.coords
    J = np.empty(X.shape + (3, 3))
    for d, C in enumerate((X, Y, Z)):
        for m, g in enumerate(op.grad_ref(pr.D, C)):
            J[..., d, m] = g
    Jinv = np.linalg.inv(J)
    Mbad = np.einsum("...dm,...dn->...mn", Jinv, Jinv)
    wq = np.einsum("k,j,i->kji", pr.w, pr.w, pr.w)[None] * np.linalg.det(J)
    Gbad = np.stack([wq * Mbad[..., a, b] for a, b in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))], 1)
    K = brute.element_matrices(pr.coords, pr.xi, pr.w, N)
    A = brute.assemble_dense(K, pr.gid, n_unique(nx, ny, nz, N))
    lattice = workload.random_lattice(22, nx, ny, nz, N, zero_boundary=False)
    u = workload.lattice_to_lvector(lattice, nx, ny, nz, N)
    Au = (pr.mask * pr.dssum(op.ax_local(u, pr.D, Gbad))).reshape(-1)
    ref = (A @ lattice.reshape(-1))[pr.gid]
    interior = pr.mask.reshape(-1) > 0
    assert np.max(np.abs(Au[interior] - ref[interior])) > 1e-8 * np.max(np.abs(ref))


@pytest.mark.parametrize("center", [0, 5, 17, 35])
def test_patch_equals_full_mesh(center):
    """The sampled-element route used at large sizes reproduces the full mesh."""
    nx, ny, nz, N = 4, 3, 3, 4
    pr = _problem(nx, ny, nz, N, 0.05)
    u = workload.continuous_rhs(1, nx, ny, nz, N, zero_boundary=False)
    P = op.Patch(nx, ny, nz, N, 0.05, center)
    n3 = (N + 1) ** 3
    up = np.concatenate([u[e * n3:(e + 1) * n3] for e in P.elements])
    for mode, ref in (("masked", pr.ax(u)), ("local", pr.ax_local(u)),
                      ("assembled", pr.ax_assembled(u))):
        assert np.array_equal(P.ax_center(up, mode), ref[center])


def test_lattice_layout_matches_element_loop():
    """The input generator's strided copy puts lattice node (ex*N+i, ey*N+j,
    ez*N+k) at element ex + nx(ey + ny ez), local (i, j, k)."""
    nx, ny, nz, N = 3, 2, 4, 3
    g = workload.random_lattice(3, nx, ny, nz, N, zero_boundary=False)
    lv = workload.lattice_to_lvector(g, nx, ny, nz, N)
    from oracle.mesh import lattice_indices
    I, J, K = lattice_indices(nx, ny, nz, N)
    assert np.array_equal(lv, g[K, J, I])
