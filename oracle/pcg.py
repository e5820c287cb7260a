"""Jacobi-preconditioned conjugate gradients in element-local storage.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Nekbone solves its Poisson problem with Jacobi (diagonally) preconditioned CG
for a fixed number of iterations, 100 by default (Sec. VIII-A).  Vectors are
kept in element-local ("L") storage, continuous across shared nodes; inner
products carry the inverse-multiplicity weight c so that every global node
counts once: <x, y>_c = sum_i c_i x_i y_i.

Iteration (x_0 = 0):
    r = b; z = Minv r; p = z; rho = <r, z>_c
    repeat:
        w = A p;  alpha = rho / <p, w>_c
        x += alpha p;  r -= alpha w
        stop if the iteration budget is spent, or (tolerance mode)
             ||r||_c <= rtol ||b||_c
        z = Minv r;  rho' = <r, z>_c;  beta = rho' / rho;  p = z + beta p
"""

from __future__ import annotations

import math

import numpy as np

from .dots import dot_c


def pcg(apply_A, b, minv, c, fixed_iter=0, rtol=1e-8, max_iter=20000, dot=dot_c,
        history=False):
    """Return (x, info) with info = dict(iters, rel_res, converged, res_hist).

    ``fixed_iter > 0`` runs exactly that many iterations (no tolerance test);
    otherwise iterate until ||r||_c <= rtol ||b||_c on the recursive residual
    or ``max_iter`` is reached.  ``rel_res`` is the recursive residual ratio.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    z = minv * r
    p = z.copy()
    rho = dot(r, z, c)
    bnorm = math.sqrt(dot(b, b, c))
    hist = []
    iters = 0
    converged = False
    limit = fixed_iter if fixed_iter > 0 else max_iter
    rnorm = bnorm
    if bnorm == 0.0:
        return x, dict(iters=0, rel_res=0.0, converged=True, res_hist=hist)
    while iters < limit:
        w = apply_A(p)
        pap = dot(p, w, c)
        alpha = rho / pap
        x += alpha * p
        r -= alpha * w
        iters += 1
        rnorm = math.sqrt(dot(r, r, c))
        if history:
            hist.append(rnorm / bnorm)
        if fixed_iter <= 0 and rnorm <= rtol * bnorm:
            converged = True
            break
        z = minv * r
        rho_new = dot(r, z, c)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    if fixed_iter > 0:
        converged = True
    return x, dict(iters=iters, rel_res=rnorm / bnorm, converged=converged, res_hist=hist)


def true_rel_residual(apply_A, b, x, c, dot=dot_c) -> float:
    """||b - A x||_c / ||b||_c."""
    r = b - apply_A(x)
    return math.sqrt(dot(r, r, c)) / math.sqrt(dot(b, b, c))
