"""Dot products for the CG reductions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The CG dot products are tree reductions in the paper (Sec. VIII-B); the
oracle instead returns the exactly rounded value, so that any summation order
on the GPU can be measured against it.

``dot_exact`` splits every product error-free (Dekker's TwoProduct with
Veltkamp's splitting; Python 3.10 has no ``math.fma``) and hands all the
pieces to ``math.fsum`` (Shewchuk's exactly rounded summation).  A weight is
applied the same way: w*x*y = (p + e)*y with p + e = w*x exactly.
"""

from __future__ import annotations

import math

import numpy as np

_SPLIT = 134217729.0  # 2**27 + 1


def _split(a):
    c = _SPLIT * a
    hi = c - (c - a)
    return hi, a - hi


def two_product(a, b):
    """p + e == a * b exactly (barring overflow/underflow)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def dot_exact(x, y, wt=None) -> float:
    """Correctly rounded sum_i (wt_i) x_i y_i."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    if wt is None:
        p, e = two_product(x, y)
        return math.fsum(np.concatenate([p, e]).tolist())
    wt = np.asarray(wt, dtype=np.float64).reshape(-1)
    p1, e1 = two_product(wt, x)
    a, b = two_product(p1, y)
    c, d = two_product(e1, y)
    return math.fsum(np.concatenate([a, b, c, d]).tolist())


def abs_sum(x, y, wt=None) -> float:
    """sum_i |wt_i x_i y_i|, the scale against which a dot's error is judged."""
    x = np.asarray(x, dtype=np.float64).reshape(-1)
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    v = np.abs(x * y)
    if wt is not None:
        v = v * np.abs(np.asarray(wt, dtype=np.float64).reshape(-1))
    return float(math.fsum(v.tolist()))


def dot_c(x, y, c) -> float:
    """sum_i c_i x_i y_i with NumPy's pairwise summation (fast; used inside
    the oracle's CG, where the iterate tolerance is far above its error)."""
    return float(np.sum(np.asarray(c).reshape(-1) * np.asarray(x).reshape(-1) * np.asarray(y).reshape(-1)))
