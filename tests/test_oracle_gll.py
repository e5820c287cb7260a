"""Pins of the oracle's GLL nodes, weights and derivative matrix.

Each check comes from outside the oracle: textbook closed forms, 50-digit
roots of P_N' from mpmath, exactness of quadrature and differentiation on
polynomials, and two other constructions of D.
"""

import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle.gll import deriv_matrix, gll_nodes_weights, legendre
from oracle.brute import vandermonde_deriv


CLOSED = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("N", sorted(CLOSED))
def test_gll_closed_forms(N):
    x, w = gll_nodes_weights(N)
    xc, wc = CLOSED[N]
    np.testing.assert_allclose(x, xc, rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, wc, rtol=4e-16, atol=0)


def _legendre_coeffs_mp(N):
    P0 = [mpmath.mpf(1)]
    P1 = [mpmath.mpf(0), mpmath.mpf(1)]
    for n in range(1, N):
        a = [mpmath.mpf(0)] + [(2 * n + 1) * c for c in P1]
        b = [n * c for c in P0] + [0, 0]
        P0, P1 = P1, [(u - v) / (n + 1) for u, v in zip(a, b)]
    return P1


@pytest.mark.parametrize("N", range(2, 16))
def test_gll_nodes_vs_mpmath(N):
    """Interior nodes are the roots of P_N'; weights 2/(N(N+1)P_N^2), at 50 digits."""
    with mpmath.workdps(50):
        c = _legendre_coeffs_mp(N)
        d = [k * c[k] for k in range(1, len(c))]
        roots = sorted(mpmath.re(r) for r in mpmath.polyroots(d[::-1], maxsteps=300, extraprec=300))
        nodes = [mpmath.mpf(-1)] + roots + [mpmath.mpf(1)]
        weights = []
        for r in nodes:
            pN = mpmath.polyval(c[::-1], r)
            weights.append(2 / (N * (N + 1) * pN * pN))
        xr = np.array([float(v) for v in nodes])
        wr = np.array([float(v) for v in weights])
    x, w = gll_nodes_weights(N)
    ulp = np.spacing(1.0)
    assert np.max(np.abs(x - xr)) <= 2 * ulp
    # w = 2 / (N (N+1) P_N^2) with P_N from an N-step recurrence: its rounding
    # grows with N (about one ulp per step, twice for the square), so above the
    # built orders the bound is 2N ulp
    assert np.max(np.abs(w - wr) / wr) <= (8 if N <= 12 else 2 * N) * ulp


@pytest.mark.parametrize("N", range(1, 16))
def test_gll_quadrature_exactness(N):
    x, w = gll_nodes_weights(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 2e-14, k
    # Lobatto quadrature is not exact at degree 2N (a defining property); the
    # defect shrinks fast with N (3e-9 at N = 15), still far above rounding
    k = 2 * N
    assert abs(np.sum(w * x ** k) - 2.0 / (k + 1)) > (1e-8 if N <= 12 else 1e-12)


def test_deriv_closed_forms():
    np.testing.assert_allclose(deriv_matrix(1), [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-15)
    np.testing.assert_allclose(deriv_matrix(2), [[-1.5, 2.0, -0.5], [-0.5, 0.0, 0.5], [0.5, -2.0, 1.5]],
                               atol=1e-15)


@pytest.mark.parametrize("N", range(1, 16))
def test_deriv_exact_on_polynomials(N):
    x, _ = gll_nodes_weights(N)
    D = deriv_matrix(N)
    scale = np.max(np.abs(D))
    for k in range(N + 1):
        d = D @ x ** k
        exact = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        assert np.max(np.abs(d - exact)) <= 1e-12 * scale * max(1, k), (N, k)


@pytest.mark.parametrize("N", range(1, 16))
def test_deriv_three_routes_agree(N):
    """Barycentric (oracle) vs the Legendre closed form
    D_ij = P_N(x_i)/(P_N(x_j)(x_i-x_j)), D_00 = -N(N+1)/4, D_NN = N(N+1)/4,
    vs the Legendre-Vandermonde route V' V^-1."""
    x, _ = gll_nodes_weights(N)
    D = deriv_matrix(N)
    pN, _ = legendre(N, x)
    n = N + 1
    DL = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                DL[i, j] = pN[i] / (pN[j] * (x[i] - x[j]))
    DL[0, 0] = -N * (N + 1) / 4
    DL[N, N] = N * (N + 1) / 4
    scale = np.max(np.abs(D))
    assert np.max(np.abs(D - DL)) <= 1e-13 * scale
    assert np.max(np.abs(D - vandermonde_deriv(x, N))) <= 1e-12 * scale


def test_stiffness_1d_closed_forms():
    for N, K in ((1, [[0.5, -0.5], [-0.5, 0.5]]),
                 (2, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 6.0)):
        _, w = gll_nodes_weights(N)
        D = deriv_matrix(N)
        np.testing.assert_allclose(D.T @ np.diag(w) @ D, K, atol=1e-14)


def test_legendre_recurrence_values():
    """P_3(x) = (5x^3 - 3x)/2 and P_4(x) = (35x^4 - 30x^2 + 3)/8 exactly at
    rational points (fractions keep the reference exact)."""
    for xv in (Fraction(1, 3), Fraction(-2, 7), Fraction(5, 9)):
        p4, p3 = legendre(4, float(xv))
        e3 = (5 * xv ** 3 - 3 * xv) / 2
        e4 = (35 * xv ** 4 - 30 * xv ** 2 + 3) / 8
        assert abs(float(p3) - float(e3)) < 1e-15
        assert abs(float(p4) - float(e4)) < 1e-15
