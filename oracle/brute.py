"""Dense brute-force element and global stiffness matrices for tiny meshes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

An independent route to the same operator as :mod:`oracle.operator`: the
1-D derivative matrix comes from a Legendre-Vandermonde basis change
(D = V' V^{-1}), the three reference derivatives are dense Kronecker
products, the metric inverse is the explicit adjugate formula, and the
element matrices K_e = sum_mn B_m^T diag(G_mn) B_n are assembled into a dense
global matrix over unique nodes.  Cost is O((N+1)^9) per element: N <= 4 and
a few elements only.
"""

from __future__ import annotations

import numpy as np


def legendre_vandermonde(x, N):
    """V_ij = P_j(x_i) and V'_ij = P_j'(x_i) for j = 0..N, using
    P'_{n+1} = P'_{n-1} + (2n+1) P_n."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    V = np.zeros((n, N + 1))
    dV = np.zeros((n, N + 1))
    V[:, 0] = 1.0
    if N >= 1:
        V[:, 1] = x
        dV[:, 1] = 1.0
    for k in range(1, N):
        V[:, k + 1] = ((2 * k + 1) * x * V[:, k] - k * V[:, k - 1]) / (k + 1)
        dV[:, k + 1] = dV[:, k - 1] + (2 * k + 1) * V[:, k]
    return V, dV


def vandermonde_deriv(x, N):
    V, dV = legendre_vandermonde(x, N)
    return dV @ np.linalg.inv(V)


def ref_derivative_ops(Dv):
    """Dense r, s, t derivative matrices on element vectors flattened [k, j, i]."""
    n = Dv.shape[0]
    I = np.eye(n)
    Br = np.kron(I, np.kron(I, Dv))
    Bs = np.kron(I, np.kron(Dv, I))
    Bt = np.kron(Dv, np.kron(I, I))
    return Br, Bs, Bt


def inverse_3x3_adjugate(J):
    """Inverse of every 3x3 matrix in J[..., 3, 3] from the adjugate, plus det."""
    a, b, c = J[..., 0, 0], J[..., 0, 1], J[..., 0, 2]
    d, e, f = J[..., 1, 0], J[..., 1, 1], J[..., 1, 2]
    g, h, k = J[..., 2, 0], J[..., 2, 1], J[..., 2, 2]
    A = e * k - f * h
    B = -(d * k - f * g)
    C = d * h - e * g
    det = a * A + b * B + c * C
    inv = np.empty_like(J)
    inv[..., 0, 0] = A
    inv[..., 1, 0] = B
    inv[..., 2, 0] = C
    inv[..., 0, 1] = -(b * k - c * h)
    inv[..., 1, 1] = a * k - c * g
    inv[..., 2, 1] = -(a * h - b * g)
    inv[..., 0, 2] = b * f - c * e
    inv[..., 1, 2] = -(a * f - c * d)
    inv[..., 2, 2] = a * e - b * d
    return inv / det[..., None, None], det


def element_matrices(coords, xi, w, N):
    """Dense element stiffness matrices, shape (E, n^3, n^3)."""
    X, Y, Z = coords
    E = X.shape[0]
    n = N + 1
    Dv = vandermonde_deriv(xi, N)
    Bops = ref_derivative_ops(Dv)
    wq = np.kron(w, np.kron(w, w))  # flattened [k, j, i] weight w_k w_j w_i
    K = np.zeros((E, n ** 3, n ** 3))
    for e in range(E):
        J = np.zeros((n ** 3, 3, 3))
        for d, C in enumerate((X, Y, Z)):
            cf = C[e].reshape(-1)
            for m in range(3):
                J[:, d, m] = Bops[m] @ cf
        Jinv, det = inverse_3x3_adjugate(J)
        for m in range(3):
            for q in range(3):
                g = wq * det * np.sum(Jinv[:, m, :] * Jinv[:, q, :], axis=1)
                K[e] += Bops[m].T @ (g[:, None] * Bops[q])
    return K


def assemble_dense(K, gid, n_glob):
    """Global matrix sum_e P_e^T K_e P_e over unique ids."""
    A = np.zeros((n_glob, n_glob))
    E, m, _ = K.shape
    g = gid.reshape(E, m)
    for e in range(E):
        A[np.ix_(g[e], g[e])] += K[e]
    return A
