"""Pins of the oracle's exact dot products and low-precision emulation."""

from fractions import Fraction

import numpy as np
import pytest
import torch

import workload
from oracle import operator as op, pcg as opcg
from oracle.dots import abs_sum, dot_exact, two_product
from oracle.mixed import (ax_local_abs_bound, ax_local_rounded, inner_outer, round_bf16,
                          round_f32)


def _fraction_dot(x, y, w=None):
    s = Fraction(0)
    for i in range(len(x)):
        t = Fraction(float(x[i])) * Fraction(float(y[i]))
        if w is not None:
            t *= Fraction(float(w[i]))
        s += t
    return s


@pytest.mark.parametrize("n,seed", [(1, 0), (17, 1), (1000, 2)])
def test_dot_exact_vs_fractions(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, n) * 10.0 ** rng.integers(-8, 8, n)
    y = rng.uniform(-1, 1, n)
    w = rng.choice([1.0, 0.5, 0.25, 0.125], n)
    assert dot_exact(x, y) == float(_fraction_dot(x, y))
    assert dot_exact(x, y, w) == float(_fraction_dot(x, y, w))
    # non-power-of-two weights take the full error-free route
    w2 = rng.uniform(0.1, 3.0, n)
    assert dot_exact(x, y, w2) == float(_fraction_dot(x, y, w2))


def test_dot_exact_heavy_cancellation():
    x = np.array([1e16, 1.0, -1e16, 3.0])
    y = np.ones(4)
    assert dot_exact(x, y) == 4.0
    assert abs_sum(x, y) == 2e16 + 4.0


def test_two_product_is_error_free():
    rng = np.random.default_rng(3)
    a = rng.uniform(-1e3, 1e3, 200)
    b = rng.uniform(-1e-3, 1e-3, 200)
    p, e = two_product(a, b)
    for i in range(200):
        assert Fraction(float(p[i])) + Fraction(float(e[i])) == Fraction(float(a[i])) * Fraction(float(b[i]))


def test_round_bf16_matches_torch():
    """torch's CPU float32 -> bfloat16 cast rounds to nearest even."""
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(-4, 4, 5000), rng.standard_normal(5000) * 1e-5,
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(round_bf16(x), ref)
    assert np.array_equal(round_f32(x), x.astype(np.float32).astype(np.float64))


def test_rounded_operator_reduces_to_fp64():
    pr = op.Problem(2, 2, 2, 5, 0.05)
    u = workload.iid_lvector(8, pr.L)
    assert np.array_equal(ax_local_rounded(pr, u, "f64"), pr.ax_local(u))
    # the rounded operators sit within their rounding bound of the exact one
    exact = pr.ax_local(u)
    # (u, D, G rounded: 3 roundings per product, plus the bfloat16 rounding of
    # the weighted gradient in that mode)
    for prec, eps, k in (("f32", 2.0 ** -24, 4), ("bf16", 2.0 ** -8, 6)):
        diff = np.abs(ax_local_rounded(pr, u, prec) - exact)
        bound = ax_local_abs_bound(pr, u, prec)
        assert np.all(diff <= k * eps * bound + 1e-300)
        # and the rounding is really there (a rounded operator is not exact)
        assert np.max(diff) > 0.01 * eps * np.max(bound)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_inner_outer_reaches_fp64_solution(prec):
    nx = ny = nz = 2
    N = 5
    pr = op.Problem(nx, ny, nz, N, 0.05)
    b = pr.shape4(workload.continuous_rhs(9, nx, ny, nz, N))
    x, info = inner_outer(pr, b, prec, rtol=1e-8)
    assert info["converged"], info
    x64, i64 = opcg.pcg(pr.ax, b, pr.minv, pr.c, rtol=1e-12)
    tr = opcg.true_rel_residual(pr.ax, b, pr.shape4(x), pr.c)
    assert tr <= 1e-8
    err = np.max(np.abs(x - x64.reshape(-1))) / np.max(np.abs(x64))
    assert err < 1e-6
