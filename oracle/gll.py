"""Gauss-Lobatto-Legendre nodes, weights and the 1-D derivative matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's SEM kernels depend on derivative matrices that depend only on the
polynomial order N (Sec. III) and on N as the bound of the 1d-dof loops
(Sec. VIII-B).  The nodal basis is the Lagrange basis on the N+1 GLL points.
"""

from __future__ import annotations

import numpy as np


def legendre(N: int, x):
    """Return (P_N(x), P_{N-1}(x)) by the three-term recurrence
    (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if N == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    for n in range(1, N):
        p_prev, p = p, ((2 * n + 1) * x * p - n * p_prev) / (n + 1)
    return p, p_prev


def gll_nodes_weights(N: int):
    """GLL nodes xi_0 < ... < xi_N on [-1, 1] and quadrature weights.

    xi_0 = -1, xi_N = 1; the interior nodes are the roots of P_N'.  Newton's
    method is applied to q(x) = (1 - x^2) P_N'(x) = N (P_{N-1}(x) - x P_N(x)),
    whose derivative is -N (N+1) P_N(x) by Legendre's equation, from the
    Chebyshev-Gauss-Lobatto guesses -cos(pi i / N).  Weights are
    w_i = 2 / (N (N+1) P_N(xi_i)^2).
    """
    if N < 1:
        raise ValueError("order N must be >= 1")
    x = -np.cos(np.pi * np.arange(N + 1) / N)
    interior = x[1:-1].copy()
    for _ in range(100):
        p, pm = legendre(N, interior)
        dx = (pm - interior * p) / ((N + 1) * p)
        interior = interior + dx
        if np.all(np.abs(dx) < 1e-16):
            break
    for _ in range(2):
        p, pm = legendre(N, interior)
        interior = interior + (pm - interior * p) / ((N + 1) * p)
    x[1:-1] = interior
    x[0], x[-1] = -1.0, 1.0
    # The node set is symmetric about 0.
    x = 0.5 * (x - x[::-1])
    if N % 2 == 0:
        x[N // 2] = 0.0
    pN, _ = legendre(N, x)
    w = 2.0 / (N * (N + 1) * pN * pN)
    return x, w


def barycentric_weights(x):
    """lambda_j = 1 / prod_{k != j} (x_j - x_k)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    lam = np.ones(n)
    for j in range(n):
        for k in range(n):
            if k != j:
                lam[j] /= (x[j] - x[k])
    return lam


def deriv_matrix(N: int, x=None):
    """D_ij = l_j'(xi_i), the derivative of the j-th Lagrange basis polynomial
    at node i, in barycentric form (Berrut & Trefethen 2004):
    D_ij = (lambda_j / lambda_i) / (x_i - x_j) for i != j, and the diagonal is
    the negative row sum (the derivative of a constant is zero)."""
    if x is None:
        x, _ = gll_nodes_weights(N)
    lam = barycentric_weights(x)
    n = len(x)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D
