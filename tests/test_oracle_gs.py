"""Pins of the oracle's generic gather-scatter (the compressed-row ``gs`` of
paper Sec. V-B) against what holds independently of its row loop: the dense
0/1 copy matrix Q (Q Q^T v), exact integer sums, closed-form counts of a
periodic box, and the box mesh's own global ids."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import gs, mesh, operator as op


def dense_q(gid):
    """Q[i, g] = 1 when L entry i is a copy of global id g."""
    uniq, inv = np.unique(gid, return_inverse=True)
    Q = np.zeros((gid.size, uniq.size))
    Q[np.arange(gid.size), inv] = 1.0
    return Q


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gs_equals_dense_qqt_on_random_ids(seed):
    rng = np.random.default_rng(seed)
    n = 300
    gid = rng.integers(0, 90, n)
    v = rng.uniform(-1, 1, n)
    off, ids = gs.csr_from_ids(gid)
    Q = dense_q(gid)
    np.testing.assert_allclose(gs.gs_csr(v, off, ids), Q @ (Q.T @ v), rtol=0, atol=1e-14)


def test_gs_integer_values_exact_and_structure():
    rng = np.random.default_rng(7)
    n = 500
    gid = rng.integers(0, 200, n)
    v = rng.integers(-1000, 1000, n).astype(np.float64)
    off, ids = gs.csr_from_ids(gid)
    out = gs.gs_csr(v, off, ids)
    # exact sums, computed with rationals
    sums = {}
    for g, x in zip(gid, v):
        sums[g] = sums.get(g, Fraction(0)) + Fraction(x)
    assert all(Fraction(out[i]) == sums[gid[i]] for i in range(n))
    # structure: every row has >= 2 copies of one id, rows ascend by id,
    # copies ascend by L index, and rows + singletons cover every entry once
    counts = np.bincount(gid)
    lens = np.diff(off)
    assert (lens >= 2).all()
    row_ids = [gid[ids[a]] for a in off[:-1]]
    assert row_ids == sorted(row_ids) and len(set(row_ids)) == len(row_ids)
    for r in range(len(lens)):
        m = ids[off[r]:off[r + 1]]
        assert (np.diff(m) > 0).all() and (gid[m] == gid[m[0]]).all()
    assert lens.sum() + (counts == 1).sum() == n
    assert len(row_ids) == (counts >= 2).sum()


def test_gs_edge_cases():
    # no shared id: no rows, vector unchanged
    off, ids = gs.csr_from_ids(np.arange(10))
    assert off.tolist() == [0] and ids.size == 0
    # one id everywhere: one row holding every entry
    off, ids = gs.csr_from_ids(np.zeros(6, dtype=np.int64))
    assert off.tolist() == [0, 6] and ids.tolist() == list(range(6))
    out = gs.gs_csr(np.arange(6, dtype=np.float64), off, ids)
    assert (out == 15.0).all()
    # empty input
    off, ids = gs.csr_from_ids(np.zeros(0, dtype=np.int64))
    assert off.tolist() == [0] and ids.size == 0


@pytest.mark.parametrize("nx,ny,nz,N", [(2, 3, 2, 3), (3, 3, 3, 2), (1, 2, 2, 4)])
def test_non_periodic_ids_match_box_mesh(nx, ny, nz, N):
    g = gs.periodic_global_ids(nx, ny, nz, N, periodic=(False, False, False))
    assert (g == mesh.global_ids(nx, ny, nz, N)).all()


@pytest.mark.parametrize("nx,ny,nz,N", [(2, 3, 2, 3), (3, 2, 4, 2)])
def test_periodic_box_counts_and_multiplicity(nx, ny, nz, N):
    g = gs.periodic_global_ids(nx, ny, nz, N)
    # a fully periodic lattice has nx*N * ny*N * nz*N distinct nodes
    assert np.unique(g).size == nx * N * ny * N * nz * N
    mult = op.multiplicity(g)
    # every element node has multiplicity 2^(number of its local coordinates on
    # the element's boundary): 8 at corners, 4 on edges, 2 on faces, 1 inside
    n = N + 1
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    on = lambda a: ((a == 0) | (a == N)).astype(int)
    expect = 2.0 ** (on(i) + on(j) + on(k)).reshape(-1)
    assert (mult.reshape(-1, n ** 3) == expect[None]).all()
    # sum of inverse multiplicities counts the distinct nodes exactly
    assert np.sum(1.0 / mult) == pytest.approx(nx * N * ny * N * nz * N, rel=0, abs=1e-9)


def test_periodic_gs_of_continuous_periodic_field():
    nx, ny, nz, N = 2, 2, 3, 3
    g = gs.periodic_global_ids(nx, ny, nz, N)
    vals = np.random.default_rng(3).uniform(-1, 1, int(g.max()) + 1)
    u = vals[g]  # continuous on the periodic lattice
    off, ids = gs.csr_from_ids(g)
    np.testing.assert_allclose(gs.gs_csr(u, off, ids), op.multiplicity(g) * u, rtol=1e-15)


def _gs_mutant(kind):
    """Plausible mistakes in the row loop of the gather-scatter."""
    def f(v, offsets, ids):
        out = np.array(v, dtype=np.float64, copy=True)
        for r in range(len(offsets) - 1):
            members = ids[offsets[r]:offsets[r + 1]]
            if kind == "drop_last":
                s = float(np.sum(v[members[:-1]]))
            elif kind == "off_by_one":
                s = float(np.sum(v[ids[offsets[r]:offsets[r + 1] - 1]])) + v[members[0]]
            else:  # "first_only": the sum is written to the first copy only
                s = float(np.sum(v[members]))
                out[members[0]] = s
                continue
            out[members] = s
        return out
    return f


@pytest.mark.parametrize("kind", ["drop_last", "off_by_one", "first_only"])
def test_planted_gs_mistakes_are_caught(kind):
    rng = np.random.default_rng(5)
    gid = rng.integers(0, 60, 200)
    v = rng.uniform(-1, 1, 200)
    off, ids = gs.csr_from_ids(gid)
    Q = dense_q(gid)
    out = _gs_mutant(kind)(v, off, ids)
    assert np.max(np.abs(out - Q @ (Q.T @ v))) > 1e-12
