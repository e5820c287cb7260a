"""Pins of the oracle's deformed box mesh (oracle.mesh.box_coords with
amp != 0) and of the isoparametric geometry built on it.

The map is x_d = X_d + a s(X) for d = 1, 2, 3 with
s(X) = sin(2 pi X1) sin(2 pi X2) sin(2 pi X3) at the undeformed point X.
Two facts from outside the oracle fix it:

1. Hand-computed node positions.  At lattice points where every sine is 0 or
   +-1 (or +-sqrt(2)/2) the deformed position is a number one writes down:
   the undeformed (1/4, 1/4, 1/4) moves to (0.30, 0.30, 0.30), (3/4, 1/4, 1/4)
   to (0.70, 0.20, 0.20), (1/8, 1/4, 3/8) to (0.15, 0.275, 0.40).
2. The analytic Jacobian.  dx/dX = I + a 1 (grad s)^T, a rank-one update of
   the identity, so det(dx/dX) = 1 + a (s_1 + s_2 + s_3) (matrix determinant
   lemma); with the affine reference map X = X0 + (h/2)(r + 1) the Jacobian
   with respect to r is (dx/dX) diag(h/2).  The isoparametric Jacobian (D
   applied to nodal coordinates) and the metric G built from it must converge
   to these spectrally in N.

Planted mistakes in copies of box_coords (the sine's period, the bump on one
coordinate only, the bump evaluated at the deformed point, a sign) must fail
these pins.
"""

import math

import numpy as np
import pytest

from oracle import operator as op
from oracle.gll import deriv_matrix, gll_nodes_weights
from oracle.mesh import box_coords, lattice_indices

AMP = 0.05


def _node(coords, lat, nx, ny, nz, N, I, J, K):
    """Deformed position of the global lattice node (I, J, K) (first copy)."""
    LI, LJ, LK = lat
    hit = np.argwhere((LI == I) & (LJ == J) & (LK == K))
    assert hit.size, (I, J, K)
    e, k, j, i = hit[0]
    return tuple(float(c[e, k, j, i]) for c in coords)


# Lattice nodes of a 4x4x4 box at N = 2: X = I / 8.
HAND = [
    # lattice node (I, J, K) at X = (I, J, K) / 8, its deformed position
    ((2, 2, 2), (0.30, 0.30, 0.30)),          # s = 1
    ((6, 2, 2), (0.70, 0.20, 0.20)),          # s = -1
    ((6, 6, 2), (0.80, 0.80, 0.30)),          # s = (-1)(-1)(1)
    ((6, 6, 6), (0.70, 0.70, 0.70)),          # s = -1
    ((1, 2, 3), (0.15, 0.275, 0.40)),         # s = (sqrt2/2)(1)(sqrt2/2) = 1/2
    ((4, 2, 2), (0.50, 0.25, 0.25)),          # sin(pi) = 0: unmoved
    ((0, 2, 2), (0.00, 0.25, 0.25)),          # on the box face: unmoved
    # s = (sqrt2/2)(-sqrt2/2)(-sqrt2/2) = sqrt2/4, a s = 0.0125 sqrt2
    ((3, 5, 7), tuple(v + 0.0125 * math.sqrt(2.0) for v in (0.375, 0.625, 0.875))),
]


def _hand_value(I, J, K):
    """Deformed position from the map written out for the lattice point
    X = (I, J, K) / 8 with exact sines of multiples of pi/4."""
    X = np.array([I, J, K]) / 8.0
    r2 = math.sqrt(2.0) / 2.0
    table = {0: 0.0, 1: r2, 2: 1.0, 3: r2, 4: 0.0, 5: -r2, 6: -1.0, 7: -r2, 8: 0.0}
    s = table[I] * table[J] * table[K]
    return tuple(X + AMP * s)


@pytest.mark.parametrize("IJK,expect", HAND)
def test_deformed_nodes_hand_values(IJK, expect):
    nx = ny = nz = 4
    N = 2
    coords = box_coords(nx, ny, nz, N, AMP)
    lat = lattice_indices(nx, ny, nz, N)
    got = _node(coords, lat, nx, ny, nz, N, *IJK)
    assert np.allclose(got, expect, rtol=0, atol=4e-16), (got, expect)


def test_deformed_nodes_every_lattice_point_against_sine_table():
    """Every node of the 4x4x4 N = 2 box (X = I/8) equals X + a s(X) with the
    sines of multiples of pi/4 taken from a table."""
    nx = ny = nz = 4
    N = 2
    X, Y, Z = box_coords(nx, ny, nz, N, AMP)
    LI, LJ, LK = lattice_indices(nx, ny, nz, N)
    for e, k, j, i in np.ndindex(X.shape):
        ref = _hand_value(LI[e, k, j, i], LJ[e, k, j, i], LK[e, k, j, i])
        got = (X[e, k, j, i], Y[e, k, j, i], Z[e, k, j, i])
        assert max(abs(a - b) for a, b in zip(got, ref)) <= 4e-16


def _analytic_geometry(nx, ny, nz, N, amp):
    """detJ and G from the analytic Jacobian of the map at the GLL nodes."""
    xi, w = gll_nodes_weights(N)
    X0, Y0, Z0 = box_coords(nx, ny, nz, N, 0.0, xi)
    tp = 2.0 * np.pi
    sx, sy, sz = np.sin(tp * X0), np.sin(tp * Y0), np.sin(tp * Z0)
    cx, cy, cz = np.cos(tp * X0), np.cos(tp * Y0), np.cos(tp * Z0)
    grad = np.stack([tp * cx * sy * sz, tp * sx * cy * sz, tp * sx * sy * cz], axis=-1)
    F = np.broadcast_to(np.eye(3), X0.shape + (3, 3)).copy()
    F += amp * grad[..., None, :]  # dx_d/dX_m = delta_dm + a ds/dX_m (every row d)
    scale = np.array([0.5 / nx, 0.5 / ny, 0.5 / nz])
    Jr = F * scale[None, None, None, None, None, :]
    det_lemma = (1.0 + amp * grad.sum(-1)) * scale.prod()
    Jinv = np.linalg.inv(Jr)
    M = np.einsum("...md,...nd->...mn", Jinv, Jinv)
    wq = np.einsum("k,j,i->kji", w, w, w)[None] * det_lemma
    G = np.stack([wq * M[..., a, b] for a, b in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))], 1)
    return det_lemma, np.linalg.det(Jr), G


@pytest.mark.parametrize("nx,ny,nz", [(2, 2, 2), (3, 2, 4)])
def test_isoparametric_jacobian_converges_to_analytic(nx, ny, nz):
    errs_det, errs_g = [], []
    for N in (4, 6, 8, 10, 12):
        pr = op.Problem(nx, ny, nz, N, AMP)
        det_an, det_direct, G_an = _analytic_geometry(nx, ny, nz, N, AMP)
        # the determinant lemma agrees with a direct determinant of the analytic J
        assert np.max(np.abs(det_an - det_direct)) <= 1e-14 * np.max(np.abs(det_an))
        errs_det.append(np.max(np.abs(pr.detJ - det_an)) / np.max(np.abs(det_an)))
        errs_g.append(np.max(np.abs(pr.G - G_an)) / np.max(np.abs(G_an)))
    # spectral: every two orders the error falls by a large factor, down to
    # far below any algebraic rate at N = 12
    for errs in (errs_det, errs_g):
        for a, b in zip(errs, errs[1:]):
            assert b < a / 8, errs
    assert errs_det[-1] < 1e-9 and errs_g[-1] < 1e-9, (errs_det, errs_g)


# ---------------------------------------------------------------------------
# Planted mistakes in copies of box_coords.

def _coords_mutant(kind, nx, ny, nz, N, amp):
    X, Y, Z = box_coords(nx, ny, nz, N, 0.0)
    tp = 2.0 * np.pi
    if kind == "half_period":
        s = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
        return X + amp * s, Y + amp * s, Z + amp * s
    s = np.sin(tp * X) * np.sin(tp * Y) * np.sin(tp * Z)
    if kind == "x_only":
        return X + amp * s, Y, Z
    if kind == "at_deformed_point":
        Xd, Yd, Zd = X + amp * s, Y + amp * s, Z + amp * s
        s2 = np.sin(tp * Xd) * np.sin(tp * Yd) * np.sin(tp * Zd)
        return X + amp * s2, Y + amp * s2, Z + amp * s2
    if kind == "sign":
        return X - amp * s, Y - amp * s, Z - amp * s
    raise ValueError(kind)


KINDS = ["half_period", "x_only", "at_deformed_point", "sign"]


@pytest.mark.parametrize("kind", KINDS)
def test_planted_deformation_mistakes_fail_hand_values(kind):
    nx = ny = nz = 4
    N = 2
    X, Y, Z = _coords_mutant(kind, nx, ny, nz, N, AMP)
    LI, LJ, LK = lattice_indices(nx, ny, nz, N)
    worst = 0.0
    for e, k, j, i in np.ndindex(X.shape):
        ref = _hand_value(LI[e, k, j, i], LJ[e, k, j, i], LK[e, k, j, i])
        got = (X[e, k, j, i], Y[e, k, j, i], Z[e, k, j, i])
        worst = max(worst, max(abs(a - b) for a, b in zip(got, ref)))
    assert worst > 1e-3, kind


@pytest.mark.parametrize("kind", KINDS)
def test_planted_deformation_mistakes_fail_analytic_jacobian(kind):
    nx, ny, nz, N = 2, 2, 2, 10
    xi, w = gll_nodes_weights(N)
    D = deriv_matrix(N, xi)
    X, Y, Z = _coords_mutant(kind, nx, ny, nz, N, AMP)
    G, detJ = op.geometric_factors(X, Y, Z, D, w)
    det_an, _, G_an = _analytic_geometry(nx, ny, nz, N, AMP)
    err = max(np.max(np.abs(detJ - det_an)) / np.max(np.abs(det_an)),
              np.max(np.abs(G - G_an)) / np.max(np.abs(G_an)))
    assert err > 1e-3, (kind, err)
