"""Consistency of the stored oracle reference solves (tests/golden/), which
the GPU tests compare the benchmarked solve with: the files were written by
tests/golden/make_cg_golden.py from the oracle alone; here their contents are
checked against each other and against the stopping rule they record."""

import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
STEMS = [f[:-5] for f in sorted(os.listdir(GOLDEN)) if f.startswith("cg_box") and f.endswith(".json")]


def test_the_benchmarked_problem_has_a_reference():
    assert "cg_box32_n7" in STEMS


@pytest.mark.parametrize("stem", STEMS)
def test_reference_is_consistent(stem):
    with open(os.path.join(GOLDEN, stem + ".json")) as fh:
        g = json.load(fh)
    n, N, rtol = g["n"], g["N"], g["rtol"]
    assert stem == f"cg_box{n}_n{N}"
    assert g["E"] == n ** 3 and g["L"] == g["E"] * (N + 1) ** 3
    hist = g["res_hist"]
    # the recursive residual history ends at the first ratio below rtol
    assert g["converged"] and len(hist) == g["iters"] > 0
    assert hist[-1] <= rtol and all(h > rtol for h in hist[:-1])
    assert abs(hist[-1] - g["rel_res_recursive"]) <= 1e-15
    # the true residual of the stored solve meets the tolerance (reading of the criterion)
    assert g["true_rel_res"] <= rtol * (1 + 1e-3)
    xs = np.load(os.path.join(GOLDEN, g["x_samples_file"]))
    assert list(xs["elements"]) == g["sample_elements"]
    assert xs["x"].shape == (len(g["sample_elements"]), N + 1, N + 1, N + 1)
    assert np.all(np.isfinite(xs["x"]))
    assert 0 < g["b_norm_c"] and 0 < g["x_norm_c"]
