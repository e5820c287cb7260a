"""Generic gather-scatter over an arbitrary map of L-vector entries to global ids.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's ``gs`` kernel (Sec. V-B, Fig. kernel_transform) loops over the
unique ids of the shared nodes and, for each, over that id's copies: it sums
the copies and writes the sum back to every copy.  Here the id -> copies map is
held in compressed-row form:

    offsets[r] .. offsets[r+1]-1   the positions in ``ids`` of row r's copies
    ids[q]                         an L-vector index

Only ids with at least two copies get a row; rows are in ascending id order
and the copies of a row in ascending L-index order.  An entry whose id occurs
once is its own sum and is left untouched.

Unlike the box mesh's ``global_ids``, the map here may be anything: a periodic
box (ids wrap around), or random ids.  The result is the plain definition
Q Q^T v of direct stiffness summation, with Q the 0/1 matrix that copies global
values to L entries.
"""

import numpy as np


def csr_from_ids(gid):
    """Rows of the shared ids (at least two copies), ascending id; each row's
    copies in ascending L-index order.  Returns (offsets int32, ids int32)."""
    gid = np.asarray(gid, dtype=np.int64).reshape(-1)
    order = np.argsort(gid, kind="stable")  # stable: equal ids keep L order
    offsets, ids = [0], []
    q = 0
    n = gid.size
    while q < n:
        g = gid[order[q]]
        end = q
        while end < n and gid[order[end]] == g:
            end += 1
        if end - q >= 2:
            ids.extend(int(i) for i in order[q:end])
            offsets.append(len(ids))
        q = end
    return np.asarray(offsets, dtype=np.int32), np.asarray(ids, dtype=np.int32)


def gs_csr(v, offsets, ids):
    """Apply the gather-scatter row by row: every copy of a row receives the
    sum of the row's copies, added in the row's order starting from 0."""
    out = np.array(v, dtype=np.float64, copy=True).reshape(-1)
    src = np.asarray(v, dtype=np.float64).reshape(-1)
    for r in range(len(offsets) - 1):
        members = ids[offsets[r]:offsets[r + 1]]
        s = 0.0
        for i in members:
            s += src[i]
        for i in members:
            out[i] = s
    return out.reshape(np.shape(v))


def periodic_global_ids(nx, ny, nz, N, periodic=(True, True, True)):
    """Global ids of a box mesh whose opposite faces are identified in the
    directions flagged ``periodic``: lattice coordinate I along such a
    direction is taken modulo n_d*N, so the last layer of nodes coincides
    with the first.  Flattened to L = E*(N+1)^3 in the usual element-major
    order (element e = ex + nx*(ey + ny*ez), node i fastest)."""
    n = N + 1
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # element-major: e = ex + nx*(ey + ny*ez)
    ex = ex.transpose(2, 1, 0).reshape(-1)
    ey = ey.transpose(2, 1, 0).reshape(-1)
    ez = ez.transpose(2, 1, 0).reshape(-1)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    I = ex[:, None, None, None] * N + i[None]
    J = ey[:, None, None, None] * N + j[None]
    K = ez[:, None, None, None] * N + k[None]
    NX, NY, NZ = nx * N, ny * N, nz * N
    if periodic[0]:
        I = I % NX
    if periodic[1]:
        J = J % NY
    if periodic[2]:
        K = K % NZ
    SX = NX if periodic[0] else NX + 1
    SY = NY if periodic[1] else NY + 1
    return (I + SX * (J + SY * K)).reshape(-1).astype(np.int64)
