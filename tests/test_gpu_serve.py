"""GPU test of the serving form: Poisson arrivals served with continuous
batching; every served solution equals the same request solved alone
(FP64: bit for bit; mixed precision: bit for bit as well, checked within the
stated 1e-6 relative tolerance first), and all requests converge."""

import math
import os

import pytest
import torch

import workload

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2606_12650_amd as sem
    from paper_2606_12650_amd.serve import make_requests, serve, serve_per_request

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"[gpu-test] {os.environ.get('PYTEST_CURRENT_TEST', '')}", flush=True)


def _alone(req, mixed):
    A = sem.SemOperator(req.nx, req.ny, req.nz, req.N, req.amp, lowprec=mixed, device=DEV)
    b = workload.continuous_rhs_device(req.rhs_seed, req.nx, req.ny, req.nz, req.N, DEV)
    x, r = A.cg(b, rtol=1e-8, mixed=mixed is not None)
    return x, r, A


@pytest.mark.parametrize("mixed", [None, "f32", "bf16"])
def test_served_equals_alone(mixed):
    specs = workload.serving_requests(11, 24, e_lo=8, e_hi=200, orders=(3, 5, 7))
    reqs = make_requests(specs, workload.poisson_arrivals(11, 400.0, 24))
    stats, sols = serve(reqs, DEV, mixed=mixed, hbm_budget=1 << 30, max_slots=8, iters_per_step=6,
                        keep_solutions=True)
    s = stats.summary()
    print(f"[serve] mixed={mixed}: {s}")
    assert s["completed"] == 24 and s["converged"] == 24 and s["rejected"] == 0
    assert s["max_active"] > 1  # requests overlapped on the device
    c_all = {}
    for req in reqs:
        x_alone, r, A = _alone(req, mixed)
        x = sols[req.index]
        c = A.export(sem._lib.SEM_FIELD_C)
        rel = math.sqrt(float((c * (x - x_alone) ** 2).sum()) / float((c * x_alone ** 2).sum()))
        assert rel <= 1e-6, (req.index, rel)
        c_all[req.index] = torch.equal(x, x_alone)
    assert all(c_all.values()), [k for k, v in c_all.items() if not v]


def test_budget_caps_admission():
    specs = workload.serving_requests(12, 10, e_lo=8, e_hi=64, orders=(5,))
    reqs = make_requests(specs, [0.0] * 10)
    # a budget that holds the largest request beside the smallest, far less
    # than all ten together: admission must wait for memory, never exceed it
    from paper_2606_12650_amd.sem import workspace_bytes
    fp = [workspace_bytes(r.nx, r.ny, r.nz, r.N, r.amp, "f32") + 16 * r.L + 512 for r in reqs]
    budget = max(fp) + min(fp)
    assert sum(fp) > budget
    stats, _ = serve(reqs, DEV, mixed="f32", hbm_budget=budget, max_slots=8, iters_per_step=5)
    s = stats.summary()
    print(f"[serve] budget {budget}: {s}")
    assert s["converged"] == 10 and s["rejected"] == 0
    assert s["peak_bytes"] <= budget and 1 <= s["max_active"] < 10


def test_per_request_baseline_runs():
    specs = workload.serving_requests(13, 6, e_lo=8, e_hi=64, orders=(5, 7))
    reqs = make_requests(specs, workload.poisson_arrivals(13, 1000.0, 6))
    stats = serve_per_request(reqs, DEV)
    assert stats.summary()["converged"] == 6
