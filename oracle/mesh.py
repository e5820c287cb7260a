"""Box mesh of hexahedral spectral elements: coordinates, global ids, mask.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Nekbone's domain is a 3-D box split into E hexahedra, each carrying (N+1)^3
nodes of an order-N tensor basis; shared nodes are duplicated in element
storage, so about E*N^3 nodes are unique (Sec. VIII-A).

Readings (the paper gives no geometry): the box is [0,1]^3 split into
nx*ny*nz equal elements; an optional smooth deformation adds
amp*sin(2 pi X)sin(2 pi Y)sin(2 pi Z), evaluated at the undeformed point, to
all three coordinates; every face of the box carries a homogeneous Dirichlet
condition.
"""

from __future__ import annotations

import numpy as np

from .gll import gll_nodes_weights


def element_index(ex, ey, ez, nx, ny):
    return ex + nx * (ey + ny * ez)


def element_coords(e: int, nx: int, ny: int):
    """(ex, ey, ez) of element e = ex + nx*(ey + ny*ez)."""
    return e % nx, (e // nx) % ny, e // (nx * ny)


def box_coords(nx: int, ny: int, nz: int, N: int, amp: float = 0.0, xi=None, elements=None):
    """Nodal coordinates, three arrays of shape (E, N+1, N+1, N+1) indexed
    [e, k, j, i].  Node (i,j,k) of element (ex,ey,ez) sits at
    ((ex + (xi_i+1)/2)/nx, (ey + (xi_j+1)/2)/ny, (ez + (xi_k+1)/2)/nz) before the
    deformation.  With ``elements`` only those elements, in that order."""
    if xi is None:
        xi, _ = gll_nodes_weights(N)
    n = N + 1
    elems = range(nx * ny * nz) if elements is None else list(elements)
    E = len(elems)
    X = np.empty((E, n, n, n))
    Y = np.empty((E, n, n, n))
    Z = np.empty((E, n, n, n))
    t = (xi + 1.0) / 2.0
    for slot, e in enumerate(elems):
        ex, ey, ez = element_coords(e, nx, ny)
        X[slot] = ((ex + t) / nx)[None, None, :]
        Y[slot] = ((ey + t) / ny)[None, :, None]
        Z[slot] = ((ez + t) / nz)[:, None, None]
    if amp != 0.0:
        bump = amp * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(2 * np.pi * Z)
        X, Y, Z = X + bump, Y + bump, Z + bump
    return X, Y, Z


def lattice_indices(nx: int, ny: int, nz: int, N: int, elements=None):
    """Global lattice coordinates (I, J, K) of every element-local node, each of
    shape (E, N+1, N+1, N+1): I = ex*N + i, J = ey*N + j, K = ez*N + k.
    With ``elements`` only those elements, in that order."""
    n = N + 1
    elems = range(nx * ny * nz) if elements is None else list(elements)
    E = len(elems)
    I = np.empty((E, n, n, n), dtype=np.int64)
    J = np.empty_like(I)
    K = np.empty_like(I)
    ar = np.arange(n)
    for slot, e in enumerate(elems):
        ex, ey, ez = element_coords(e, nx, ny)
        I[slot] = (ex * N + ar)[None, None, :]
        J[slot] = (ey * N + ar)[None, :, None]
        K[slot] = (ez * N + ar)[:, None, None]
    return I, J, K


def global_ids(nx: int, ny: int, nz: int, N: int, elements=None):
    """Unique global id g = I + (nx*N+1)*(J + (ny*N+1)*K) of each local node,
    flattened to length L = E*(N+1)^3 (or only the listed elements)."""
    I, J, K = lattice_indices(nx, ny, nz, N, elements)
    NX, NY = nx * N + 1, ny * N + 1
    return (I + NX * (J + NY * K)).reshape(-1)


def n_unique(nx: int, ny: int, nz: int, N: int) -> int:
    return (nx * N + 1) * (ny * N + 1) * (nz * N + 1)


def dirichlet_mask(nx: int, ny: int, nz: int, N: int, elements=None):
    """1.0 at nodes strictly inside the box, 0.0 at nodes on any box face;
    flattened to length L (or only the listed elements)."""
    I, J, K = lattice_indices(nx, ny, nz, N, elements)
    on = (I == 0) | (I == nx * N) | (J == 0) | (J == ny * N) | (K == 0) | (K == nz * N)
    return np.where(on, 0.0, 1.0).reshape(-1)
