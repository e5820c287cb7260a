"""Geometric factors, the element Poisson operator, direct stiffness summation
and the Jacobi diagonal.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's most expensive kernel, ``ax``, applies the Poisson operator
element by element with N as the 1d-dof loop bound (Sec. VIII-B); elements
are independent (Sec. III); the ``gs`` kernel sums the copies of each shared
node (Sec. V-B, Fig. kernel_transform).  The formulas are those of the
collocated GLL spectral-element stiffness operator:

    A u = mask o Q Q^T A_L u,
    (A_L u)_e = sum_{m,n} D_m^T diag(G_mn) D_n u_e,

with D_r, D_s, D_t the 1-D derivative matrix applied along r, s, t and
G = w_i w_j w_k det(J) J^{-1} J^{-T} at each node.  Arrays are indexed
[e, k, j, i] (i is the r direction).
"""

from __future__ import annotations

import numpy as np

from .gll import deriv_matrix, gll_nodes_weights
from .mesh import box_coords, dirichlet_mask, global_ids

# Order of the six stored factors of the symmetric 3x3 matrix G.
FACTOR_NAMES = ("rr", "rs", "rt", "ss", "st", "tt")


def grad_ref(D, f):
    """Reference-space gradient of nodal values f[e,k,j,i]:
    (f_r, f_s, f_t) = (sum_l D_il f_eklj... along r, along s, along t)."""
    fr = np.einsum("il,ekjl->ekji", D, f)
    fs = np.einsum("jl,ekli->ekji", D, f)
    ft = np.einsum("kl,elji->ekji", D, f)
    return fr, fs, ft


def geometric_factors(X, Y, Z, D, w):
    """Isoparametric metric terms.

    J[d][m] = dx_d/dr_m is D applied along r_m to the nodal coordinate x_d.
    Returns (G, detJ): G of shape (E, 6, n, n, n) ordered rr, rs, rt, ss, st, tt
    with G_mn = w_i w_j w_k detJ sum_d (J^-1)_md (J^-1)_nd.
    """
    J = np.empty(X.shape + (3, 3))
    for d, C in enumerate((X, Y, Z)):
        cr, cs, ct = grad_ref(D, C)
        J[..., d, 0] = cr
        J[..., d, 1] = cs
        J[..., d, 2] = ct
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)  # Jinv[..., m, d] = dr_m / dx_d
    M = np.einsum("...md,...nd->...mn", Jinv, Jinv)
    wq = np.einsum("k,j,i->kji", w, w, w)
    scale = wq[None] * detJ
    G = np.empty((X.shape[0], 6) + X.shape[1:])
    for idx, (m, n) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
        G[:, idx] = scale * M[..., m, n]
    return G, detJ


def ax_local(u, D, G):
    """w = A_L u by sum factorisation: gradient along r, s, t; multiply by the
    symmetric 3x3 factor at every node; apply D^T along r, s, t and add."""
    ur, us, ut = grad_ref(D, u)
    grr, grs, grt, gss, gst, gtt = (G[:, q] for q in range(6))
    wr = grr * ur + grs * us + grt * ut
    ws = grs * ur + gss * us + gst * ut
    wt = grt * ur + gst * us + gtt * ut
    out = np.einsum("li,ekjl->ekji", D, wr)
    out += np.einsum("lj,ekli->ekji", D, ws)
    out += np.einsum("lk,elji->ekji", D, wt)
    return out


def dssum(v, gid):
    """Direct stiffness summation Q Q^T v: every copy of a global node receives
    the sum of all its copies, added in ascending element-local index order."""
    flat = np.asarray(v, dtype=np.float64).reshape(-1)
    order = np.argsort(gid, kind="stable")
    sums = np.zeros(int(gid.max()) + 1)
    for idx in order:
        sums[gid[idx]] += flat[idx]
    return sums[gid].reshape(np.shape(v))


def dssum_fast(v, gid):
    """Same sums as :func:`dssum` via ``np.add.at`` (unbuffered, applied in
    index order), for the larger meshes of the tests."""
    flat = np.asarray(v, dtype=np.float64).reshape(-1)
    sums = np.zeros(int(gid.max()) + 1)
    np.add.at(sums, gid, flat)
    return sums[gid].reshape(np.shape(v))


def multiplicity(gid):
    """Number of element-local copies of each node's global id (per L entry)."""
    counts = np.bincount(gid)
    return counts[gid].astype(np.float64)


def jacobi_diag_local(D, G):
    """Diagonal of A_L: for node (i,j,k)
    sum_l D_li^2 G_rr(l,j,k) + sum_l D_lj^2 G_ss(i,l,k) + sum_l D_lk^2 G_tt(i,j,l)
    + 2 D_ii D_jj G_rs + 2 D_ii D_kk G_rt + 2 D_jj D_kk G_st (all at (i,j,k))."""
    D2 = D * D
    grr, grs, grt, gss, gst, gtt = (G[:, q] for q in range(6))
    d = np.einsum("li,ekjl->ekji", D2, grr)
    d += np.einsum("lj,ekli->ekji", D2, gss)
    d += np.einsum("lk,elji->ekji", D2, gtt)
    dd = np.diag(D)
    di = dd[None, None, None, :]
    dj = dd[None, None, :, None]
    dk = dd[None, :, None, None]
    d += 2 * di * dj * grs + 2 * di * dk * grt + 2 * dj * dk * gst
    return d


class Problem:
    """Everything the oracle needs for one box mesh: D, w, G, gid, mask,
    multiplicity weights c = 1/mult and the Jacobi inverse diagonal."""

    def __init__(self, nx, ny, nz, N, amp=0.0, fast_dssum=True):
        self.nx, self.ny, self.nz, self.N, self.amp = nx, ny, nz, N, amp
        self.n = N + 1
        self.E = nx * ny * nz
        self.L = self.E * self.n ** 3
        self.xi, self.w = gll_nodes_weights(N)
        self.D = deriv_matrix(N, self.xi)
        X, Y, Z = box_coords(nx, ny, nz, N, amp, self.xi)
        self.coords = (X, Y, Z)
        self.G, self.detJ = geometric_factors(X, Y, Z, self.D, self.w)
        self.gid = global_ids(nx, ny, nz, N)
        self.mask = dirichlet_mask(nx, ny, nz, N).reshape(self.E, self.n, self.n, self.n)
        self._dss = dssum_fast if fast_dssum else dssum
        self.mult = multiplicity(self.gid).reshape(self.mask.shape)
        self.c = 1.0 / self.mult
        dg = self._dss(jacobi_diag_local(self.D, self.G), self.gid)
        self.diag = dg
        self.minv = np.where(self.mask > 0, 1.0 / dg, 0.0)

    def shape4(self, v):
        return np.asarray(v, dtype=np.float64).reshape(self.E, self.n, self.n, self.n)

    def ax_local(self, u):
        return ax_local(self.shape4(u), self.D, self.G)

    def ax_assembled(self, u):
        return self._dss(self.ax_local(u), self.gid)

    def ax(self, u):
        """A u = mask o dssum(A_L u)."""
        return self.mask * self.ax_assembled(u)

    def dssum(self, v):
        return self._dss(self.shape4(v), self.gid)


class Patch:
    """An element and its (up to 26) neighbours in a large box mesh.

    Every copy of a node of the centre element lies in the patch, so the
    assembled, masked operator at the centre element's nodes can be evaluated
    from the patch alone: this is how large meshes are checked at sampled
    elements without building the whole mesh.
    """

    def __init__(self, nx, ny, nz, N, amp, center):
        from .mesh import box_coords, dirichlet_mask, element_coords, global_ids
        self.N, self.n = N, N + 1
        ex, ey, ez = element_coords(center, nx, ny)
        elems = []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    a, b, c = ex + dx, ey + dy, ez + dz
                    if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
                        elems.append(a + nx * (b + ny * c))
        self.elements = sorted(elems)
        self.center_slot = self.elements.index(center)
        self.xi, self.w = gll_nodes_weights(N)
        self.D = deriv_matrix(N, self.xi)
        X, Y, Z = box_coords(nx, ny, nz, N, amp, self.xi, self.elements)
        self.G, self.detJ = geometric_factors(X, Y, Z, self.D, self.w)
        self.gid = global_ids(nx, ny, nz, N, self.elements)
        n3 = self.n ** 3
        self.mask_center = dirichlet_mask(nx, ny, nz, N, [center]).reshape(self.n, self.n, self.n)
        self.center_gid = self.gid[self.center_slot * n3:(self.center_slot + 1) * n3]

    def ax_center(self, u_patch, mode="masked"):
        """A_L, dssum(A_L) or mask o dssum(A_L) of u_patch at the centre
        element's nodes; u_patch has the patch elements' L entries in order."""
        n = self.n
        wl = ax_local(np.asarray(u_patch, dtype=np.float64).reshape(-1, n, n, n), self.D, self.G)
        if mode == "local":
            return wl[self.center_slot]
        flat = wl.reshape(-1)
        sums = {}
        for idx in np.argsort(self.gid, kind="stable"):
            g = int(self.gid[idx])
            sums[g] = sums.get(g, 0.0) + flat[idx]
        out = np.array([sums[int(g)] for g in self.center_gid]).reshape(n, n, n)
        if mode == "masked":
            out = out * self.mask_center
        return out
