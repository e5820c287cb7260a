"""Write the oracle's reference solve of a large box mesh for the GPU tests.

Runs only the FP64 oracle (``oracle/``) on inputs from ``workload`` and stores
what a GPU solve of the same problem is compared with: the Jacobi-PCG
iteration count to the relative tolerance, the recursive residual history,
the oracle's true relative residual ||b - A x||_c / ||b||_c, the c-norms of b
and x, and x on a few sampled elements.

The problem is the Nekbone Poisson solve (Sec. VIII-A): a box of
n x n x n hexahedra of order N on [0,1]^3 with the smooth deformation
x += amp sin(2 pi X) sin(2 pi Y) sin(2 pi Z), homogeneous Dirichlet data on
every face, a continuous uniform[-1, 1] right-hand side drawn per global node
(seeded), x_0 = 0, stopping at ||r||_c <= rtol ||b||_c.

The element operator A_L is block-diagonal over elements, so each operator
application evaluates the oracle's ax_local on contiguous element ranges in
a thread pool and concatenates them (the first application is checked to be
bitwise equal to the oracle's whole-mesh evaluation); the gather-scatter and
mask are the oracle's.

Usage (CPU only; the 32^3 N = 7 case takes about 40 minutes, 16^3 at N = 11 about 20):
    python tests/golden/make_cg_golden.py --N 7
    python tests/golden/make_cg_golden.py --n 16 --N 11
Outputs tests/golden/cg_box{n}_n{N}.json and tests/golden/cg_box{n}_n{N}_x.npz.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workload  # noqa: E402
from oracle import operator as op  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from oracle.dots import dot_c  # noqa: E402


def sample_elements(n: int, count: int, seed: int) -> list[int]:
    """Corner, face, edge and centre elements plus seeded random ones."""
    E = n ** 3
    h = n // 2
    fixed = [0, n - 1, E - 1, h + n * (h + n * h), h + n * (h + n * 0), 0 + n * (h + n * h)]
    rng = np.random.default_rng(seed)
    extra = [int(e) for e in rng.choice(E, size=max(0, count - len(fixed)), replace=False)]
    out = []
    for e in fixed + extra:
        if e not in out:
            out.append(e)
    return sorted(out)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=32, help="elements per direction")
    ap.add_argument("--N", type=int, default=7, help="polynomial order")
    ap.add_argument("--amp", type=float, default=0.05)
    ap.add_argument("--seed", type=int, default=4, help="right-hand side seed")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--samples", type=int, default=10, help="elements whose x is stored")
    ap.add_argument("--out", default=HERE)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1,
                    help="element ranges evaluated in parallel per operator application")
    a = ap.parse_args(argv)

    n, N = a.n, a.N
    t0 = time.time()
    pr = op.Problem(n, n, n, N, a.amp)
    print(f"[golden] setup {time.time() - t0:.1f} s (E={pr.E}, N={N}, L={pr.L})", flush=True)
    b = pr.shape4(workload.continuous_rhs(a.seed, n, n, n, N))

    pool = ThreadPoolExecutor(max(1, a.threads))
    cuts = np.linspace(0, pr.E, max(1, a.threads) + 1).astype(int)
    ranges = [(lo, hi) for lo, hi in zip(cuts[:-1], cuts[1:]) if hi > lo]

    def ax_ranges(p):
        p4 = pr.shape4(p)
        parts = pool.map(lambda r: op.ax_local(p4[r[0]:r[1]], pr.D, pr.G[r[0]:r[1]]), ranges)
        return pr.mask * op.dssum_fast(np.concatenate(list(parts)), pr.gid)

    assert np.array_equal(ax_ranges(b), pr.ax(b)), "element-range evaluation differs from the oracle"

    calls = [0]
    t1 = time.time()

    def apply_A(p):
        calls[0] += 1
        if calls[0] % 100 == 0:
            el = time.time() - t1
            print(f"[golden] {calls[0]} operator applications, {el:.0f} s", flush=True)
        return ax_ranges(p)

    x, info = opcg.pcg(apply_A, b, pr.minv, pr.c, rtol=a.rtol, history=True)
    t_solve = time.time() - t1
    true_rel = opcg.true_rel_residual(pr.ax, b, x, pr.c)
    bnorm = math.sqrt(dot_c(b, b, pr.c))
    xnorm = math.sqrt(dot_c(x, x, pr.c))
    print(f"[golden] {info['iters']} iterations in {t_solve:.0f} s, recursive {info['rel_res']:.3e}, "
          f"true {true_rel:.3e}", flush=True)

    elems = sample_elements(n, a.samples, seed=11 + N)
    xs = np.stack([x[e] for e in elems])
    stem = f"cg_box{n}_n{N}"
    meta = {
        "written_by": "tests/golden/make_cg_golden.py (FP64 oracle only)",
        "problem": "Jacobi-PCG for the Poisson problem of Sec. VIII-A on a box of n^3 hexahedra",
        "n": n, "N": N, "E": pr.E, "L": pr.L, "amp": a.amp, "rhs_seed": a.seed, "rtol": a.rtol,
        "rhs": "workload.continuous_rhs(seed, n, n, n, N): uniform[-1,1] per global node, 0 on the boundary",
        "iters": int(info["iters"]),
        "converged": bool(info["converged"]),
        "rel_res_recursive": float(info["rel_res"]),
        "true_rel_res": float(true_rel),
        "b_norm_c": bnorm,
        "x_norm_c": xnorm,
        "res_hist": [float(v) for v in info["res_hist"]],
        "sample_elements": elems,
        "x_samples_file": stem + "_x.npz",
        "oracle_solve_s": round(t_solve, 1),
    }
    with open(os.path.join(a.out, stem + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")
    np.savez_compressed(os.path.join(a.out, stem + "_x.npz"), elements=np.array(elems), x=xs)
    print(f"[golden] wrote {stem}.json and {stem}_x.npz", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
