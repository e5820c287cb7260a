"""Low-precision operator emulation and inner-outer (iterative refinement) CG.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes no precision.  The precision form evaluates the derivative
contractions with D, G and the input rounded to FP32 or BF16 (round to nearest
even) and accumulates in FP32.  In BF16 mode both inputs of each contraction
are bfloat16 (the operand u of the gradient and the G-weighted gradient that
enters the transposed contraction), as a bfloat16 matrix-core contraction
consumes them; all products are then exact in FP32.  The operator sits inside
an inner CG whose result corrects an FP64 outer iterate:

    x = 0; r = b
    repeat until ||r||_c <= rtol ||b||_c:
        s = ||r||_c
        e = inner Jacobi-PCG on A_lo e = r / s  (FP32 vectors, FP64 dots,
            stop at relative residual eta or after max_inner iterations)
        x += s e;  r = b - A x   (FP64)

The order in which MFMA accumulates is unknown, so the oracle does not try to
match low-precision iterates bit for bit ("parity unpinned"); it evaluates the
rounded operator exactly in FP64 and bounds the accumulation error
componentwise, and it pins the FP64 outer result.
"""

from __future__ import annotations

import math

import numpy as np

from .operator import ax_local


def round_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    """Round to the nearest BF16 value (ties to even), via FP32."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def rounder(prec: str):
    return {"f64": lambda v: np.asarray(v, dtype=np.float64), "f32": round_f32, "bf16": round_bf16}[prec]


def ax_local_rounded(problem, u, prec: str):
    """A_L u evaluated in FP64 with D, G and u rounded to ``prec`` (and, in
    BF16 mode, the G-weighted gradient rounded to bfloat16 before the
    transposed contraction): the value a low-precision kernel approximates
    up to its FP32 accumulation."""
    rd = rounder(prec)
    D = rd(problem.D)
    G = rd(problem.G)
    v = rd(problem.shape4(u))
    ur = np.einsum("il,ekjl->ekji", D, v)
    us = np.einsum("jl,ekli->ekji", D, v)
    ut = np.einsum("kl,elji->ekji", D, v)
    g = [G[:, q] for q in range(6)]
    wr = g[0] * ur + g[1] * us + g[2] * ut
    ws = g[1] * ur + g[3] * us + g[4] * ut
    wt = g[2] * ur + g[4] * us + g[5] * ut
    if prec == "bf16":
        wr, ws, wt = round_bf16(wr), round_bf16(ws), round_bf16(wt)
    out = np.einsum("li,ekjl->ekji", D, wr)
    out += np.einsum("lj,ekli->ekji", D, ws)
    out += np.einsum("lk,elji->ekji", D, wt)
    return out


def ax_local_abs_bound(problem, u, prec: str):
    """Componentwise magnitude |D|^T |G| |D| |u| (with rounded operands): the
    scale of the FP32 accumulation error of a low-precision A_L u."""
    rd = rounder(prec)
    return ax_local(np.abs(rd(problem.shape4(u))), np.abs(rd(problem.D)), np.abs(rd(problem.G)))


def inner_outer(problem, b, prec: str = "f32", rtol=1e-8, eta=1e-3, max_inner=200,
                max_outer=50):
    """Iterative refinement with a restarted inner Jacobi-PCG in FP32.

    The inner operator is A_lo = mask o dssum(A_L(round(D), round(G), round(.)))
    evaluated in float32 arithmetic by NumPy; dots accumulate in FP64.
    Returns (x, info) with outer and total inner iteration counts and the final
    FP64 true relative residual.
    """
    rd = rounder(prec)
    D32 = rd(problem.D).astype(np.float32)
    G32 = rd(problem.G).astype(np.float32)
    mask = problem.mask
    c = problem.c
    minv32 = problem.minv.astype(np.float32)

    def a_lo(v32):
        v = rd(v32.astype(np.float64)).astype(np.float32)
        ur = np.einsum("il,ekjl->ekji", D32, v)
        us = np.einsum("jl,ekli->ekji", D32, v)
        ut = np.einsum("kl,elji->ekji", D32, v)
        g = [G32[:, q] for q in range(6)]
        wr = g[0] * ur + g[1] * us + g[2] * ut
        ws = g[1] * ur + g[3] * us + g[4] * ut
        wt = g[2] * ur + g[4] * us + g[5] * ut
        if prec == "bf16":
            wr, ws, wt = (rd(t.astype(np.float64)).astype(np.float32) for t in (wr, ws, wt))
        out = np.einsum("li,ekjl->ekji", D32, wr)
        out = out + np.einsum("lj,ekli->ekji", D32, ws)
        out = out + np.einsum("lk,elji->ekji", D32, wt)
        return (mask * problem.dssum(out.astype(np.float64))).astype(np.float32)

    def dot(x, y):
        return float(np.sum(c * x.astype(np.float64) * y.astype(np.float64)))

    b = problem.shape4(b)
    bnorm = math.sqrt(dot(b, b))
    x = np.zeros_like(b)
    r = b.copy()
    outer = 0
    inner_total = 0
    rel = 1.0
    while outer < max_outer:
        s = math.sqrt(dot(r, r))
        rel = s / bnorm
        if rel <= rtol:
            break
        rr = (r / s).astype(np.float32)
        e = np.zeros_like(rr)
        res = rr.copy()
        z = minv32 * res
        p = z.copy()
        rho = dot(res, z)
        r0 = math.sqrt(dot(res, res))
        for _ in range(max_inner):
            w = a_lo(p)
            alpha = rho / dot(p, w)
            e = (e + np.float32(alpha) * p).astype(np.float32)
            res = (res - np.float32(alpha) * w).astype(np.float32)
            inner_total += 1
            if math.sqrt(dot(res, res)) <= eta * r0:
                break
            z = minv32 * res
            rho_new = dot(res, z)
            p = (z + np.float32(rho_new / rho) * p).astype(np.float32)
            rho = rho_new
        x = x + s * e.astype(np.float64)
        r = b - problem.ax(x)
        outer += 1
    rel = math.sqrt(dot(r, r)) / bnorm
    return x.reshape(-1), dict(outer=outer, inner=inner_total, rel_res=rel, converged=rel <= rtol)
