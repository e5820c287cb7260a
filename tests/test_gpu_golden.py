"""Large solves against the FP64 oracle's own solves of the same problems:
the benchmarked one (32x32x32 deformed box, N = 7) and a 16x16x16 deformed
box at N = 11 (the order of the large-order workload), Jacobi-PCG to
||r||_c <= 1e-8 ||b||_c from x = 0 (Sec. VIII-A).

The oracle's solves take from half an hour to hours on a CPU, so their
results are stored: tests/golden/cg_box{n}_n{N}.json and _x.npz, written by
tests/golden/make_cg_golden.py, which runs only the oracle.

Criteria (CG iterates are not unique in finite precision; any x that meets
the residual is a correct solution):
  FP64 solve
  - iteration counts within 2 of the oracle's;
  - both true relative residuals ||b - A x||_c / ||b||_c <= 1e-8 (1 + 1e-3),
    the GPU's computed with the oracle's operator (on a stored problem above
    2e7 points, whose oracle set-up would take minutes, with the GPU's FP64
    operator, which matches the oracle's to 1e-12 in the A.u parity tests);
  - the recursive residual ratios of the first 20 iterations within 1e-6
    (relative) of the oracle's;
  - x on the sampled elements within 1e-6 (c-weighted, relative) of the
    oracle's x there.
  Inner-outer solves (FP32 and BF16 inner operators)
  - the FP64 true residual <= 1e-8 (1 + 1e-3) (GPU FP64 operator);
  - x on the sampled elements within 1e-5 of the oracle's FP64 solution
    (condition number times the tolerance).
"""

import json
import math
import os

import numpy as np
import pytest
import torch

import workload
from oracle import operator as op
from oracle import pcg as opcg
from oracle.mesh import global_ids

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2606_12650_amd as sem

DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
STEMS = [f[:-5] for f in sorted(os.listdir(GOLDEN)) if f.startswith("cg_box") and f.endswith(".json")]
ORACLE_OPERATOR_MAX_L = 20_000_000  # oracle set-up within a few seconds


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"[gpu-test] {os.environ.get('PYTEST_CURRENT_TEST', '')}", flush=True)


def _load(stem):
    with open(os.path.join(GOLDEN, stem + ".json")) as fh:
        meta = json.load(fh)
    xs = np.load(os.path.join(GOLDEN, meta["x_samples_file"]))
    return meta, xs["elements"], xs["x"]


def _sampled_rel(g, elems, xs_ref, x):
    """c-weighted relative difference of x from the oracle's on the samples."""
    n, N = g["n"], g["N"]
    n1 = N + 1
    mult = op.multiplicity(global_ids(n, n, n, N)).reshape(-1, n1, n1, n1)
    c = 1.0 / mult[elems]
    d = x.reshape(-1, n1, n1, n1)[elems] - xs_ref
    return math.sqrt(float(np.sum(c * d * d)) / float(np.sum(c * xs_ref * xs_ref)))


def _gpu_true_rel(A, g, b, x):
    """||b - A x||_c / ||b||_c with the GPU's FP64 operator (c-weighted dots
    on the host)."""
    n, N = g["n"], g["N"]
    c = 1.0 / op.multiplicity(global_ids(n, n, n, N)).reshape(-1)
    ax = A.ax(x, sem.MASKED)
    torch.cuda.synchronize()
    bh = b.cpu().numpy()  # zero on the box boundary, as A x is
    r = bh - ax.cpu().numpy()
    return math.sqrt(float(np.sum(c * r * r)) / float(np.sum(c * bh * bh)))


@pytest.mark.parametrize("stem", STEMS)
def test_solve_matches_oracle_reference(stem):
    g, elems, xs_ref = _load(stem)
    n, N, amp, rtol = g["n"], g["N"], g["amp"], g["rtol"]
    print(f"[golden] {stem}: n = {n}, N = {N}", flush=True)
    bnp = workload.continuous_rhs(g["rhs_seed"], n, n, n, N)
    A = sem.SemOperator(n, n, n, N, amp, device=DEV)
    b = torch.from_numpy(bnp).to(DEV)
    x, res = A.cg(b, rtol=rtol)
    assert res.status == 0
    print(f"[golden] GPU iterations {res.iters}, oracle {g['iters']}", flush=True)
    assert abs(res.iters - g["iters"]) <= 2
    assert g["true_rel_res"] <= rtol * (1 + 1e-3)

    # the residual history of the first 20 iterations
    x2 = torch.empty_like(b)
    for k in range(1, 21):
        _, rk = A.cg(b, x2, fixed_iter=k)
        ref = g["res_hist"][k - 1]
        assert abs(rk.rel_res - ref) <= 1e-6 * ref, (k, rk.rel_res, ref)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()

    # x on the sampled elements
    rel = _sampled_rel(g, elems, xs_ref, xg)
    print(f"[golden] x on {len(elems)} sampled elements: relative c-norm difference {rel:.3e}", flush=True)
    assert rel <= 1e-6

    # the GPU solution's true residual
    if g["L"] <= ORACLE_OPERATOR_MAX_L:
        A.close()
        del b, x, x2
        pr = op.Problem(n, n, n, N, amp)
        tr = opcg.true_rel_residual(pr.ax, pr.shape4(bnp), pr.shape4(xg), pr.c)
        how = "oracle operator"
    else:
        tr = _gpu_true_rel(A, g, b, x)
        A.close()
        how = "GPU FP64 operator"
    print(f"[golden] true relative residual of the GPU x ({how}) {tr:.3e}", flush=True)
    assert tr <= rtol * (1 + 1e-3)


@pytest.mark.parametrize("stem", STEMS)
@pytest.mark.parametrize("lowprec", ["f32", "bf16"])
def test_mixed_solve_matches_oracle_reference(stem, lowprec):
    g, elems, xs_ref = _load(stem)
    n, N, amp, rtol = g["n"], g["N"], g["amp"], g["rtol"]
    bnp = workload.continuous_rhs(g["rhs_seed"], n, n, n, N)
    A = sem.SemOperator(n, n, n, N, amp, lowprec=lowprec, device=DEV)
    b = torch.from_numpy(bnp).to(DEV)
    x, res = A.cg(b, rtol=rtol, mixed=True)
    assert res.status == 0
    tr = _gpu_true_rel(A, g, b, x)
    xg = x.cpu().numpy()
    A.close()
    rel = _sampled_rel(g, elems, xs_ref, xg)
    print(f"[golden] {stem} {lowprec}: outer {res.outer_iters}, true residual {tr:.3e}, "
          f"x vs oracle on samples {rel:.3e}", flush=True)
    assert tr <= rtol * (1 + 1e-3)
    assert rel <= 1e-5
