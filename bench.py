"""Benchmark of the spectral-element Poisson hot path on one MI355X.

Step = one Jacobi-PCG solve to ||r||_c <= 1e-8 ||b||_c from x = 0 on the
32x32x32 deformed hex mesh at N = 7 (E = 32768, 16.8 M element-local nodes),
with the operator already set up and the right-hand side resident in HBM.
Throughput is the paper's GDOFS measure (Sec. VIII-B, Eq. gdofs):
E*N^3*iterations / time / 1e9.

Beside it the bench times the A.u operator kernel alone (the roofline study of
the same mesh) with HIP events on the stream it runs on, and the FP64 CPU
oracle on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published peak
METRIC = "GDOF/s A·u and CG solves/s, mixed vs FP64 at 1e-8 rel res; p99 latency"


def _source_digest(files) -> str:
    """Hash of the kernel sources' code: comments and blank lines are left out,
    so that a comment edit keeps committed counter runs valid."""
    import re

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2606_12650_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode("utf-8"))
    return h.hexdigest()[:16]


def _kernel_source_hash() -> str:
    return _source_digest(("sem_ax.hip", "sem_ax_mfma.h", "sem_ax_tile.h", "sem_internal.h",
                           "sem_device.h", "sem_kernels.h", "sem_types.h"))


def _cg_source_hash() -> str:
    """Hash of every source the CG iteration's kernels are built from."""
    return _source_digest(("sem_ax.hip", "sem_ax_mfma.h", "sem_ax_tile.h", "sem_internal.h",
                           "sem_device.h", "sem_kernels.h", "sem_types.h", "sem_cg_dev.h",
                           "sem_vec.hip"))


def _traffic_from_profile(kernel_hash: str):
    """HBM bytes per launch of the A.u kernel from committed rocprofv3 counter
    runs, if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "ax_f64_n7_e32768_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


MFMA_PROFILE = os.path.join(ROOT, "profiles", "mfma_e32768_counters.json")


def _mfma_from_profile(kernel_hash: str, kernel: str):
    """Matrix-core use of `kernel` (a substring of its name) from the committed
    rocprofv3 counter run (MFMA ops and busy cycles), if it was taken on the
    current kernel source; else None.  Keys: dtype, mfma_flops_per_launch,
    achieved_tflops, peak_tflops, util (achieved / dense peak of the type),
    busy_frac (MFMA-busy SIMD cycles / all SIMD cycles of the launch)."""
    if not os.path.exists(MFMA_PROFILE):
        return None
    with open(MFMA_PROFILE) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    row = d.get("kernels", {}).get(kernel)
    if not row or "util" not in row:
        return None
    dt = row["dtype"]
    return {"dtype": dt, "mfma_flops_per_launch": row["mfma_flops_per_dispatch"][dt],
            "achieved_tflops": row["achieved_tflops"], "peak_tflops": row["peak_tflops"],
            "util": row["util"], "busy_frac": row["busy_frac"], "profiled_avg_us": row["avg_us"]}


def _cg_traffic_frac(iters: int, wall: float):
    """HBM bytes the CG iterations actually moved (operator and update
    kernels, from the committed counter runs, while the kernel source is
    unchanged) over the solve time, as a fraction of the peak; None without
    matching counters."""
    path = os.path.join(ROOT, "profiles", "ax_f64_n7_e32768_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("cg_source_hash") != _cg_source_hash():
        return None
    per_iter = 0.0
    for name, v in d.get("all_kernels", {}).items():
        # the CG operator and the default update tile (shape 0) of this order
        if "ax_mfma_kernel<8, semk::PrecF64, true>" in name or "cg_update_kernel<8, double, 0>" in name:
            per_iter += v["hbm_bytes"]
    if per_iter == 0.0:
        return None
    return per_iter * iters / wall / 1e9 / HBM_PEAK_GBS


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_timed(fn, reps: int):
    """Best of `reps` wall times of fn() and the cores it used (CPU time over
    wall time of the best run)."""
    best, cores = float("inf"), 1.0
    for _ in range(reps):
        t0, c0 = time.perf_counter(), time.process_time()
        fn()
        wall, cpu = time.perf_counter() - t0, time.process_time() - c0
        if wall < best:
            best, cores = wall, cpu / max(wall, 1e-9)
    return best, cores


def cpu_baseline(gpu_iters_c2: int, include_c2: bool = True):
    """The FP64 NumPy oracle, as it stands, timed on this host's cores.

    C1 (4x4x4 affine box, N = 7): one masked A.u, 50 Jacobi-PCG iterations,
    axpy and dot on 32768 entries.  C2 (the benchmarked 32x32x32 deformed box
    at N = 7): one masked A.u and three PCG iterations, the per-iteration time
    multiplied by the iteration count of the GPU solve to 1e-8 (setup
    excluded, as on the GPU).  Each at two settings: every host core allowed
    to the BLAS / OpenMP pools (OMP_NUM_THREADS = nproc), and one core.  The
    cores a setting actually used are measured (CPU time over wall time): the
    oracle's sum factorisation is NumPy einsum, which runs on one core either
    way.  Best of 3 wall times."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workload
    from oracle import operator as op
    from oracle import pcg as opcg

    nproc = os.cpu_count() or 1
    settings = {}
    N = 7
    c1 = op.Problem(4, 4, 4, N, 0.0)
    u1 = c1.shape4(workload.continuous_rhs(1, 4, 4, 4, N))
    b1 = c1.shape4(workload.continuous_rhs(2, 4, 4, 4, N))
    rng = np.random.default_rng(3)
    xa, ya = rng.uniform(-1.0, 1.0, c1.L), rng.uniform(-1.0, 1.0, c1.L)
    c2 = None
    if include_c2:
        t0 = time.perf_counter()
        c2 = op.Problem(32, 32, 32, N, 0.05)
        b2 = c2.shape4(workload.continuous_rhs(4, 32, 32, 32, N))
        c2_setup = time.perf_counter() - t0
    for label, lim in (("all_cores", nproc), ("one_core", 1)):
        with threadpool_limits(lim):
            row = {"threads_allowed": lim}
            t, cores = _cpu_timed(lambda: c1.ax(u1), 3)
            row["c1_ax_us"], row["c1_ax_cores"] = t * 1e6, cores
            t, cores = _cpu_timed(lambda: opcg.pcg(c1.ax, b1, c1.minv, c1.c, fixed_iter=50), 3)
            row["c1_pcg50_ms"], row["c1_pcg_cores"] = t * 1e3, cores
            row["c1_pcg_us_per_iter"] = t / 50 * 1e6
            t, _ = _cpu_timed(lambda: ya + 0.5 * xa, 3)
            row["c1_axpy_us"] = t * 1e6
            t, _ = _cpu_timed(lambda: float(np.dot(xa, ya)), 3)
            row["c1_dot_us"] = t * 1e6
            if c2 is not None:
                t, cores = _cpu_timed(lambda: c2.ax(b2), 2)
                row["c2_ax_s"], row["c2_ax_cores"] = t, cores
                row["c2_ax_gdofs"] = c2.E * N ** 3 / t / 1e9
                t, cores = _cpu_timed(lambda: opcg.pcg(c2.ax, b2, c2.minv, c2.c, fixed_iter=3), 1)
                per_it = t / 3
                row["c2_pcg_s_per_iter"], row["c2_pcg_cores"] = per_it, cores
                row["c2_pcg_gdofs"] = c2.E * N ** 3 / per_it / 1e9
                row["c2_solve_s_extrapolated"] = per_it * gpu_iters_c2
                row["c2_solves_per_s_extrapolated"] = 1.0 / (per_it * gpu_iters_c2)
            settings[label] = row
    main_row = settings["all_cores"]
    if c2 is not None:
        value = main_row["c2_pcg_gdofs"]
        cores_used = main_row["c2_pcg_cores"]
        sample = (f"FP64 NumPy oracle Jacobi-PCG on the benchmarked 32x32x32 deformed N=7 mesh, "
                  f"3 iterations timed (setup {c2_setup:.0f} s excluded), GDOF/s per Eq. gdofs; "
                  f"solve time = per-iteration time x {gpu_iters_c2} GPU iterations; C1 rows in 'settings'")
    else:
        value = main_row["c1_pcg50_ms"] and c1.E * N ** 3 * 50 / (main_row["c1_pcg50_ms"] / 1e3) / 1e9
        cores_used = main_row["c1_pcg_cores"]
        sample = "FP64 NumPy oracle, C1 only (4x4x4 affine N=7, 50 PCG iterations)"
    return {
        "value": value,
        "unit": "GDOF/s",
        "cores": round(cores_used, 2),
        "kind": "oracle",
        "sample": sample,
        "nproc": nproc,
        "cpu_model": _cpu_model(),
        "settings": settings,
    }


def _timed(fn):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, r


def _graph_time(fn, reps: int, stream, runs: int = 5):
    """Per-call time of fn() (a launch sequence on `stream`): `reps` calls
    captured once as a HIP graph, one untimed replay, then `runs` replays
    timed with HIP events on that stream.  Returns (mean, min) seconds per
    call over the runs."""
    import torch

    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    per = []
    for _ in range(runs):
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        g.replay()
        a1.record(stream)
        torch.cuda.synchronize()
        per.append(a0.elapsed_time(a1) / 1e3 / reps)
    del g
    return sum(per) / len(per), min(per)


# Stored bytes per element-local node of one A.u (read u and the six G
# factors, write w): FP64 8 words; FP32 4-byte words; BF16 mode u and w FP32,
# G as bfloat16.
AX_BYTES_PER_POINT = {"f64": 64.0, "f32": 32.0, "bf16": 20.0}


def _ax_kernel_name(prec: str, N: int, mfma: bool) -> str:
    P = {"f64": "PrecF64", "f32": "PrecF32", "bf16": "PrecBF16"}[prec]
    # the element-local sem_ax runs the matrix-core tile's streaming-store kernel
    return f"ax_mfma_local_kernel<{N + 1}, {P}>" if mfma else f"ax_kernel<{N + 1}, {P}, false>"


def _default_is_mfma(prec: str, N: int) -> bool:
    # the library's per-order default (sem_internal.h op_uses_mfma)
    return N >= 7 if prec in ("f64", "f32") else N >= 9


def bench_ax_study(args, dev, orders=(7, 11)) -> dict:
    """A.u alone (one element-local launch, SEM_AX_LOCAL) on the 32x32x32
    deformed mesh at each order in FP64, FP32 and BF16 mode, with the default
    element kernel of that order and precision and with the other one forced:
    microseconds per launch (graph-replayed, the paper's 5-run protocol),
    GDOF/s (E N^3 per launch) and the fraction of the 8 TB/s HBM peak on the
    stored bytes per node."""
    import torch

    import workload
    import paper_2606_12650_amd as sem

    nx = ny = nz = 32
    amp = 0.05
    out = {}
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        for N in orders:
            u64 = torch.from_numpy(workload.continuous_rhs(5, nx, ny, nz, N)).to(dev)
            u32 = u64.to(torch.float32)
            row = {}
            for prec in ("f64", "f32", "bf16"):
                dflt = _default_is_mfma(prec, N)
                for mf in (dflt, not dflt):
                    A = sem.SemOperator(nx, ny, nz, N, amp, lowprec=None if prec == "f64" else prec,
                                        device=dev, mfma=mf)
                    if prec == "f64":
                        w = torch.empty_like(u64)
                        fn = lambda: A.ax(u64, sem.LOCAL, out=w)  # noqa: E731
                    else:
                        w = torch.empty_like(u32)
                        fn = lambda: A.ax_lowp(u32, sem.LOCAL, out=w)  # noqa: E731
                    mean, best = _graph_time(fn, args.ax_reps, stream)
                    bpp = AX_BYTES_PER_POINT[prec]
                    gbs = bpp * A.L / mean / 1e9
                    key = prec if mf == dflt else prec + "_alt"
                    row[key] = {"kernel": _ax_kernel_name(prec, N, mf), "default": mf == dflt,
                                "us": mean * 1e6, "best_run_us": best * 1e6,
                                "gdofs": A.E * N ** 3 / mean / 1e9, "bytes_per_point": bpp,
                                "gbs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
                    if mf:
                        P = {"f64": "PrecF64", "f32": "PrecF32", "bf16": "PrecBF16"}[prec]
                        row[key]["mfma"] = _mfma_from_profile(_kernel_source_hash(),
                                                              f"ax_mfma_local_kernel<{N + 1}, semk::{P}>")
                    print(f"[bench] ax N={N} {key}: {row[key]}", file=sys.stderr, flush=True)
                    A.close()
                    del A, w
            row["E"] = nx * ny * nz
            row["L"] = nx * ny * nz * (N + 1) ** 3
            out[f"N{N}"] = row
            del u64, u32
    torch.cuda.synchronize()
    return out


def profile_kernels(args, dev) -> dict:
    """A short run of every kernel the counter summaries cover, for rocprofv3:
    a plain 1 GiB device copy (the calibration of the HBM counters), the A.u
    study (N = 7 and 11, FP64 / FP32 / BF16, both element tiles), and on the
    32x32x32 deformed mesh at N = 7 and 11: 50 FP64 PCG iterations and 50
    inner iterations of each mixed solver (one outer step)."""
    import torch

    import workload
    import paper_2606_12650_amd as sem

    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    out = {"ax_study": bench_ax_study(args, dev)}
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        for N in (7, 11):
            b = torch.from_numpy(workload.continuous_rhs(4, 32, 32, 32, N)).to(dev)
            A = sem.SemOperator(32, 32, 32, N, 0.05, device=dev)
            _, r = A.cg(b, fixed_iter=50, check_every=25)
            out[f"cg_n{N}_fp64_50"] = r.iters
            A.close()
            for prec in ("f32", "bf16"):
                A = sem.SemOperator(32, 32, 32, N, 0.05, lowprec=prec, device=dev)
                _, r = A.cg(b, rtol=1e-8, mixed=True, max_iter=1, inner_max=50, check_every=25,
                            raise_on_fail=False)
                out[f"cg_n{N}_{prec}_inner"] = r.iters
                A.close()
            del b
    torch.cuda.synchronize()
    return out


def bench_c1(args, dev) -> dict:
    """The small case (4x4x4 affine box, N = 7, E = 64, L = 32768; its 2 MB
    stay in the caches, so it is timed per operation, not against HBM): one
    masked A.u, one Jacobi-PCG iteration (50 fixed iterations), axpy and dot
    on 32768 entries, and the time of an empty-work launch sequence."""
    import torch

    import workload
    import paper_2606_12650_amd as sem

    nx = ny = nz = 4
    N = 7
    stream = torch.cuda.Stream(device=dev)
    out = {"E": 64, "N": N, "L": 32768}
    with torch.cuda.stream(stream):
        A = sem.SemOperator(nx, ny, nz, N, 0.0, device=dev)
        u = torch.from_numpy(workload.continuous_rhs(1, nx, ny, nz, N)).to(dev)
        b = torch.from_numpy(workload.continuous_rhs(2, nx, ny, nz, N)).to(dev)
        w = torch.empty_like(u)
        mean, _ = _graph_time(lambda: A.ax(u, sem.MASKED, out=w), 200, stream)
        out["ax_masked_us"] = mean * 1e6
        mean, _ = _graph_time(lambda: A.ax(u, sem.LOCAL, out=w), 200, stream)
        out["ax_local_us"] = mean * 1e6
        x = torch.empty_like(b)
        A.cg(b, x, fixed_iter=50, check_every=50)
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            A.cg(b, x, fixed_iter=50, check_every=50)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        out["pcg50_ms"] = sum(times) / len(times) * 1e3
        out["pcg_us_per_iter"] = out["pcg50_ms"] / 50 * 1e3
        rng = __import__("numpy").random.default_rng(3)
        xa = torch.from_numpy(rng.uniform(-1.0, 1.0, 32768)).to(dev)
        ya = torch.from_numpy(rng.uniform(-1.0, 1.0, 32768)).to(dev)
        mean, _ = _graph_time(lambda: sem.vec_axpy(0.5, xa, ya), 200, stream)
        out["axpy_us"] = mean * 1e6
        ws = sem.vec_dot_workspace(32768, dev)
        d = torch.empty(1, dtype=torch.float64, device=dev)
        mean, _ = _graph_time(lambda: sem.vec_dot(xa, ya, out=d, ws=ws), 200, stream)
        out["dot_us"] = mean * 1e6
        # launch floor: an axpy over one entry (one work-group)
        mean, _ = _graph_time(lambda: sem.vec_axpy(0.5, xa[:1], ya[:1]), 200, stream)
        out["one_workgroup_launch_us"] = mean * 1e6
        A.close()
    torch.cuda.synchronize()
    print(f"[bench] C1: {out}", file=sys.stderr, flush=True)
    return out


def bench_precision_order(args, dev, N: int) -> dict:
    """The precision study at a second order on the same 32x32x32 deformed
    mesh: FP64 PCG and the inner-outer FP32 / BF16 solves to 1e-8 with the
    default element kernels, the error of each against the FP64 solution."""
    import torch

    import workload
    import paper_2606_12650_amd as sem

    nx = ny = nz = 32
    amp, rtol = 0.05, 1e-8
    out = {"N": N}
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        b = torch.from_numpy(workload.continuous_rhs(4, nx, ny, nz, N)).to(dev)
        x64 = None
        for prec in (None, "f32", "bf16"):
            A = sem.SemOperator(nx, ny, nz, N, amp, lowprec=prec, device=dev)
            x = torch.empty_like(b)
            mixed = prec is not None
            A.cg(b, x, rtol=rtol, mixed=mixed)  # warm-up (graph capture)
            torch.cuda.synchronize()
            steps = 2
            t0 = time.perf_counter()
            for _ in range(steps):
                _, res = A.cg(b, x, rtol=rtol, mixed=mixed)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / steps
            entry = {"solves_per_s": 1.0 / wall, "ms_per_solve": wall * 1e3, "iters": res.iters,
                     "outer_iters": res.outer_iters, "rel_res_fp64": res.rel_res, "status": res.status}
            if prec is None:
                x64 = x.clone()
                c_w = A.export(sem._lib.SEM_FIELD_C)
                entry["gdofs"] = A.E * N ** 3 * res.iters / wall / 1e9
                out["fp64"] = entry
            else:
                entry["rel_err_vs_fp64_solution"] = math.sqrt(
                    float((c_w * (x - x64) ** 2).sum()) / float((c_w * x64 ** 2).sum()))
                entry["speedup_vs_fp64"] = out["fp64"]["ms_per_solve"] / entry["ms_per_solve"]
                out[prec] = entry
            print(f"[bench] precision N={N} {prec or 'fp64'}: {entry}", file=sys.stderr, flush=True)
            A.close()
            del x
    torch.cuda.synchronize()
    return out


def bench_batching(args, dev) -> dict:
    """256 independent solves (log-uniform E in [64, 4096], N in {3,5,7,9,11},
    deformed geometry, seeded right-hand sides) to 1e-8: one at a time with
    sem_cg in FP64, then all together in one batch (FP64, and inner-outer
    FP32 / BF16), with operator tiles from the autotuner."""
    import torch

    import workload
    import paper_2606_12650_amd as sem
    from paper_2606_12650_amd import autotune
    from paper_2606_12650_amd.batch import SemBatch

    specs = workload.batch_instances(seed=1000, count=args.batch_instances)
    stream = torch.cuda.Stream(device=dev)
    res = {"instances": len(specs)}
    with torch.cuda.stream(stream):
        t_tune, tiles = _timed(lambda: autotune.tune(device=dev, cache_path=None))
        res["tiles"] = {p: {str(k): v for k, v in d.items()} for p, d in tiles.items()}
        res["autotune_s"] = t_tune
        print(f"[bench] autotuned tiles {res['tiles']} in {t_tune:.1f} s", file=sys.stderr, flush=True)
        ops, rhs = [], []
        for sp in specs:
            op = sem.SemOperator(sp["nx"], sp["ny"], sp["nz"], sp["N"], sp["amp"], lowprec="f32", device=dev)
            ops.append(op)
            rhs.append(workload.continuous_rhs_device(sp["rhs_seed"], sp["nx"], sp["ny"], sp["nz"], sp["N"], dev))
        res["total_points"] = int(sum(op.L for op in ops))
        res["total_gdof"] = int(sum(op.E * op.order ** 3 for op in ops))
        xs = [op.empty() for op in ops]
        # one at a time, FP64
        def per_instance():
            its = 0
            for op, b, x in zip(ops, rhs, xs):
                _, r = op.cg(b, x, rtol=1e-8)
                its += r.iters
            return its
        per_instance()  # warm-up (graph capture per operator)
        t_seq, its_seq = _timed(per_instance)
        x_ref = [x.clone() for x in xs]
        res["fp64_per_instance"] = {"solves_per_s": len(ops) / t_seq, "wall_s": t_seq, "iters": its_seq}
        print(f"[bench] batching: per-instance FP64 {t_seq:.2f} s", file=sys.stderr, flush=True)
        for mode in ("fp64", "f32", "bf16"):
            mops = ops
            if mode == "bf16":
                mops = [sem.SemOperator(sp["nx"], sp["ny"], sp["nz"], sp["N"], sp["amp"], lowprec="bf16",
                                        device=dev) for sp in specs]
            def run_batch():
                B = SemBatch(len(mops), device=dev)
                autotune.apply(B, tiles)
                slots = [B.add(op, b, x, rtol=1e-8, mixed=(mode != "fp64")) for op, b, x in zip(mops, rhs, xs)]
                out = B.run_all(iters_per_step=20)
                for q in slots:
                    B.remove(q)
                B.close()
                return out
            run_batch()  # warm-up
            t_b, out = _timed(run_batch)
            ok = sum(1 for r in out.values() if r.status == 0 and r.rel_res <= 1e-8)
            entry = {"solves_per_s": len(mops) / t_b, "wall_s": t_b, "converged": ok,
                     "speedup_vs_fp64_per_instance": t_seq / t_b}
            if mode == "fp64":
                entry["bitwise_equal_to_per_instance"] = all(torch.equal(a, b) for a, b in zip(xs, x_ref))
            else:
                errs = []
                for op, a, b in zip(mops, xs, x_ref):
                    c = op.export(sem._lib.SEM_FIELD_C)
                    errs.append(math.sqrt(float((c * (a - b) ** 2).sum()) / float((c * b ** 2).sum())))
                entry["max_rel_err_vs_fp64"] = max(errs)
            res[f"{mode}_batched"] = entry
            print(f"[bench] batching: {mode} batched {entry}", file=sys.stderr, flush=True)
            if mode == "bf16":
                for op in mops:
                    op.close()
        for op in ops:
            op.close()
    torch.cuda.synchronize()
    return res


def bench_serving(args, dev, rates=None, n=None, warmup=None, budgets_gb=None) -> dict:
    """Poisson arrivals of solve requests (log-uniform E in [64, 32768], N in
    {5,7,9}, tolerance 1e-8; request seeds 5): continuous batching with the
    inner-outer FP32 solver under an HBM budget vs one FP64 sem_cg per
    request.  For each arrival rate: `n` timed requests after `warmup`
    untimed ones (the percentiles and the throughput window cover the timed
    ones), at each budget.  A rate is marked overload when it exceeds the
    throughput the server reached at it (the queue then grows for the whole
    run and the latencies measure its drain, not service time)."""
    import workload
    from paper_2606_12650_amd import serve as sv

    rates = rates or [float(r) for r in args.serve_rates.split(",") if r]
    n = args.serve_requests if n is None else n
    warmup = args.serve_warmup if warmup is None else warmup
    budgets_gb = budgets_gb or [32]
    out = {}
    for rate in rates:
        specs = workload.serving_requests(5, n + warmup)
        reqs = sv.make_requests(specs, workload.poisson_arrivals(5, rate, n + warmup))
        row = {}
        for gb in budgets_gb:
            st_b, _ = sv.serve(reqs, dev, mixed="f32", hbm_budget=int(gb) << 30, max_slots=64, iters_per_step=20)
            sb = st_b.summary(warmup)
            sb["overload"] = rate > 1.1 * sb["solves_per_s"]
            row["mixed_f32_continuous_batching" if gb == budgets_gb[0] else f"mixed_f32_budget_{gb}gb"] = sb
            print(f"[bench] serving rate {rate} budget {gb} GB: batched {sb['solves_per_s']:.1f}/s "
                  f"p50 {sb['p50_latency_s']:.2f}s p99 {sb['p99_latency_s']:.2f}s", file=sys.stderr, flush=True)
        st_p = sv.serve_per_request(reqs, dev)
        sp = st_p.summary(warmup)
        sp["overload"] = rate > 1.1 * sp["solves_per_s"]
        sb = row["mixed_f32_continuous_batching"]
        row["fp64_per_request"] = sp
        row["solves_per_s_ratio"] = sb["solves_per_s"] / max(sp["solves_per_s"], 1e-12)
        row["p99_ratio"] = sb["p99_latency_s"] / max(sp["p99_latency_s"], 1e-12)
        out[f"{rate:g}"] = row
        print(f"[bench] serving rate {rate}: batched {sb['solves_per_s']:.1f}/s p99 {sb['p99_latency_s']:.2f}s, "
              f"per-request {sp['solves_per_s']:.1f}/s p99 {sp['p99_latency_s']:.2f}s", file=sys.stderr, flush=True)
    out["requests_per_rate"] = n
    out["warmup_requests"] = warmup
    out["hbm_budgets_gb"] = budgets_gb
    out["mesh_mix"] = "E log-uniform [64, 32768], N uniform {5,7,9}, amp 0.05, tol 1e-8"
    return out


def serve_study(args) -> int:
    """The serving protocol of the measurement plan: arrival rates 50, 100,
    200, 500, 1000 and 2000 requests/s (all above one GPU's capacity of about
    13 solves/s at this mix, so overload) plus rates below capacity, `n`
    timed requests after `warmup`, HBM budgets 32 GB and a tighter one.
    Prints one JSON line."""
    import torch

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    rates = [float(r) for r in args.serve_study_rates.split(",") if r]
    budgets = [int(b) for b in args.serve_study_budgets.split(",") if b]
    res = bench_serving(args, dev, rates=rates, n=args.serve_requests, warmup=args.serve_warmup,
                        budgets_gb=budgets)
    print(json.dumps({"serve_study": res}), flush=True)
    return 0


def _box_for(E: int):
    """Balanced power-of-two box with E = 2^p elements."""
    p = int(round(math.log2(E)))
    dims = [1, 1, 1]
    for q in range(p):
        dims[q % 3] *= 2
    return dims[0], dims[1], dims[2]


def _specialisation_ablation(A, b, nx, ny, nz, N, stream, reps: int) -> dict:
    """The paper's HIP-fixed vs HIP-variable comparison (Sec. VIII-B,
    Tab. hip_vs_hip) per kernel on this mesh: microseconds per call, mean of 5
    graph-replayed runs of `reps` calls, of
      ax:   the operator (element-local A_L u) with N fixed at compile time
            (the vector-ALU column tile) vs the same mapping with N a
            run-time argument (sem_ax_generic);
      dot:  vec_dot (group size and unrolled tree fixed) vs vec_dot_generic
            (group size 256 chosen at launch, looped tree), n = L;
      axpy: vec_axpy (group size fixed) vs vec_axpy_generic (256 at launch).
    ``speedup`` is generic time over fixed time."""
    import torch

    import paper_2606_12650_amd as sem

    dev = b.device
    Av = sem.SemOperator(nx, ny, nz, N, 0.05, device=dev, mfma=False)
    w = torch.empty_like(b)
    y = b.clone()
    out = torch.empty(1, dtype=torch.float64, device=dev)
    ws = sem.vec_dot_workspace(A.L, dev)
    nb = int(sem._lib.lib().vec_dot_generic_workspace_bytes(A.L, 256))
    wsg = torch.empty(max(1, (nb + 7) // 8), dtype=torch.float64, device=dev)
    pairs = {
        "ax": (lambda: Av.ax(b, sem.LOCAL, out=w), lambda: Av.ax_generic(b, out=w)),
        "dot": (lambda: sem.vec_dot(b, y, out=out, ws=ws),
                lambda: sem.vec_dot_generic(b, y, out=out, ws=wsg, block=256)),
        "axpy": (lambda: sem.vec_axpy(1e-3, b, y), lambda: sem.vec_axpy_generic(1e-3, b, y, block=256)),
    }
    res = {}
    for name, (fixed, generic) in pairs.items():
        tf, _ = _graph_time(fixed, reps, stream)
        tg, _ = _graph_time(generic, reps, stream)
        res[name] = {"fixed_us": tf * 1e6, "generic_us": tg * 1e6, "speedup": tg / tf}
    Av.close()
    return res


def sweep(args) -> int:
    """GDOFS vs number of DOFs (the paper's Sec. VIII-B study, Eq. gdofs),
    re-run on one MI355X: for each N in {4, 6, 8} and E = 2^1..2^14 (balanced
    power-of-two boxes, deformed), 100 warm-up CG iterations, then 100 timed
    iterations, the time averaged over 5 runs.  The solver is the paper's
    plain (unpreconditioned) CG of its Nekbone runs (Sec. VIII-A);
    ``--sweep-pcg`` runs the Jacobi-PCG of the library's default instead.
    Each row also holds the relative residual ||r||_c / ||b||_c after the 100
    iterations, with a flag for the paper's 1e-7 .. 1e-6 band (Sec. VIII-C;
    the paper's right-hand side is not ours, so the band is context, not a
    pass mark).  One JSON line per (N, E), then one summary line."""
    import torch

    import workload
    import paper_2606_12650_amd as sem

    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    precond = bool(args.sweep_pcg)
    rows = []
    with torch.cuda.stream(stream):
        for N in (4, 6, 8):
            for p in range(1, 15):
                nx, ny, nz = _box_for(2 ** p)
                A = sem.SemOperator(nx, ny, nz, N, 0.05, device=dev)
                b = torch.from_numpy(workload.continuous_rhs(4, nx, ny, nz, N)).to(dev)
                x = torch.empty_like(b)
                A.cg(b, x, fixed_iter=100, check_every=100, precond=precond)  # warm-up (and graph capture)
                times = []
                for _ in range(5):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, res = A.cg(b, x, fixed_iter=100, check_every=100, precond=precond)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                t = sum(times) / len(times)
                E = nx * ny * nz
                row = {"N": N, "E": E, "box": [nx, ny, nz], "dofs": E * N ** 3,
                       "unique_dofs": (nx * N + 1) * (ny * N + 1) * (nz * N + 1),
                       "solver": "jacobi_pcg" if precond else "cg",
                       "t_100_iters_s": t, "t_min_s": min(times), "gdofs": E * N ** 3 * 100 / t / 1e9,
                       "rel_res_100": res.rel_res, "in_paper_band_1e-7_1e-6": 1e-7 <= res.rel_res <= 1e-6}
                if not args.no_ablation:
                    row["ablation"] = _specialisation_ablation(A, b, nx, ny, nz, N, stream, args.ax_reps)
                rows.append(row)
                print(json.dumps(row), flush=True)
                A.close()
    best = {N: max(r["gdofs"] for r in rows if r["N"] == N) for N in (4, 6, 8)}
    sat = {}
    for N in (4, 6, 8):
        rs = [r for r in rows if r["N"] == N]
        top = max(r["gdofs"] for r in rs)
        first = next((r["dofs"] for r in rs if r["gdofs"] >= 0.9 * top), None)
        sat[N] = first
    summary = {"sweep": "gdofs_vs_dofs", "solver": "jacobi_pcg" if precond else "cg",
               "max_gdofs": best, "dofs_at_90pct_of_max": sat}
    if not args.no_ablation:
        big = {N: max((r for r in rows if r["N"] == N), key=lambda r: r["E"]) for N in (4, 6, 8)}
        summary["ablation_speedup_at_largest_E"] = {
            N: {k: v["speedup"] for k, v in r["ablation"].items()} for N, r in big.items()}
    print(json.dumps(summary), flush=True)
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ax-reps", type=int, default=20, help="launches per timed run of A.u (5 runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-batch", action="store_true", help="skip the 256-instance batching study")
    ap.add_argument("--skip-serve", action="store_true", help="skip the serving study")
    ap.add_argument("--skip-n11", action="store_true", help="skip the precision study at N = 11")
    ap.add_argument("--skip-mixed", action="store_true", help="skip the mixed-precision solves at N = 7")
    ap.add_argument("--skip-ax-study", action="store_true",
                    help="skip the A.u study at N = 7 and 11 in FP64 / FP32 / BF16")
    ap.add_argument("--skip-c1", action="store_true", help="skip the small-case (4x4x4, N = 7) timings")
    ap.add_argument("--ax-only", action="store_true",
                    help="only the A.u study; prints its JSON")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="a short run of every kernel the profiles cover (for rocprofv3); prints its JSON")
    ap.add_argument("--skip-tune", action="store_true",
                    help="skip the kernel-shape search of the single-solve CG (autotune.tune_solver)")
    ap.add_argument("--tune-only", action="store_true",
                    help="only the kernel-shape search at N = 7 and 11; prints its JSON")
    ap.add_argument("--batch-instances", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=100)
    ap.add_argument("--serve-rates", type=str, default="5,50,1000",
                    help="arrival rates (requests/s) of the serving study in the default run")
    ap.add_argument("--serve-warmup", type=int, default=10,
                    help="untimed requests before the timed ones at each rate")
    ap.add_argument("--serve-study", action="store_true",
                    help="only the serving protocol (--serve-study-rates, --serve-study-budgets, "
                         "--serve-requests timed after --serve-warmup); prints its JSON")
    ap.add_argument("--serve-study-rates", type=str, default="2,5,10,50,100,200,500,1000,2000")
    ap.add_argument("--serve-study-budgets", type=str, default="32,8", help="HBM budgets in GB")
    ap.add_argument("--sweep", action="store_true",
                    help="the paper's study instead: GDOF/s vs DOFs for N = 4, 6, 8, E = 2^1..2^14, "
                         "100 warm-up + 100 timed plain CG iterations, mean of 5 runs")
    ap.add_argument("--no-ablation", action="store_true",
                    help="with --sweep: skip the fixed-vs-generic kernel timings")
    ap.add_argument("--sweep-pcg", action="store_true",
                    help="with --sweep: Jacobi-PCG instead of the paper's plain CG")
    args = ap.parse_args(argv)
    if args.sweep and args.gpus == 1:
        return sweep(args)
    if args.serve_study and args.gpus == 1:
        return serve_study(args)
    if args.tune_only and args.gpus == 1:
        import torch

        from paper_2606_12650_amd import autotune

        torch.cuda.set_device(0)
        print(json.dumps({"autotune_solver": autotune.tune_solver(orders=(7, 11), cache_path=None)}),
              flush=True)
        return 0
    if (args.ax_only or args.profile_kernels) and args.gpus == 1:
        import torch

        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        if args.profile_kernels:
            print(json.dumps(profile_kernels(args, dev)), flush=True)
        else:
            print(json.dumps({"ax_study": bench_ax_study(args, dev)}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the path is single-GPU; see the sharding notes in the design document)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import workload
    import paper_2606_12650_amd as sem

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    nx = ny = nz = 32
    N, amp, rtol = 7, 0.05, 1e-8
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        A = sem.SemOperator(nx, ny, nz, N, amp, device=dev)
        b = torch.from_numpy(workload.continuous_rhs(4, nx, ny, nz, N)).to(dev)
        x = torch.empty_like(b)
        w = torch.empty_like(b)
        torch.cuda.synchronize()
        print(f"[bench] setup done: E={A.E} N={N} L={A.L}", file=sys.stderr, flush=True)

        # ---- warm-up and timed solves
        iters = []
        for _ in range(args.warmup):
            _, res = A.cg(b, x, rtol=rtol)
            iters.append(res.iters)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        timed_iters = 0
        res = None
        for _ in range(args.steps):
            _, res = A.cg(b, x, rtol=rtol)
            timed_iters += res.iters
        ev1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        wall = t1 - t0
        ev_ms = ev0.elapsed_time(ev1)
        if res is None or res.status != 0:
            print(f"[bench] solve failed: {res}", file=sys.stderr)
            return 1
        print(f"[bench] {args.steps} solves, {timed_iters} iterations, {wall:.3f} s", file=sys.stderr,
              flush=True)

        # ---- A.u operator kernel alone (sem_ax, element-local mode: one launch)
        u = torch.from_numpy(workload.continuous_rhs(5, nx, ny, nz, N)).to(dev)
        for _ in range(3):
            A.ax(u, sem.LOCAL, out=w)
        torch.cuda.synchronize()
        # the paper's protocol (Sec. VIII-B): several timed runs of repeated
        # launches; the mean over all launches is the reported duration.  The
        # launches of a run are captured once as a HIP graph, so that host
        # time between launches (a profiler's, say) does not enter the timing.
        ax_graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(ax_graph, stream=stream):
            for _ in range(args.ax_reps):
                A.ax(u, sem.LOCAL, out=w)
        ax_graph.replay()
        torch.cuda.synchronize()
        ax_runs = []
        for _ in range(5):
            a0 = torch.cuda.Event(enable_timing=True)
            a1 = torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            ax_graph.replay()
            a1.record(stream)
            torch.cuda.synchronize()
            ax_runs.append(a0.elapsed_time(a1) / 1e3 / args.ax_reps)
        ax_s = sum(ax_runs) / len(ax_runs)
        ax_s_min = min(ax_runs)
        # masked A.u (operator + gather-scatter), the full sem_ax
        m0 = torch.cuda.Event(enable_timing=True)
        m1 = torch.cuda.Event(enable_timing=True)
        m0.record(stream)
        for _ in range(args.ax_reps):
            A.ax(u, sem.MASKED, out=w)
        m1.record(stream)
        torch.cuda.synchronize()
        axm_s = m0.elapsed_time(m1) / 1e3 / args.ax_reps

        # ---- plain device copy of a known size (reference for HBM counters)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(10):
            dst.copy_(src)
        c1.record(stream)
        torch.cuda.synchronize()
        copy_s = c0.elapsed_time(c1) / 1e3 / 10
        copy_gbs = 2 * src.numel() * 8 / copy_s / 1e9
        # this library's own streaming kernel (vec_axpy: read x and y, write y)
        sem.vec_axpy(0.5, src, dst)
        c0.record(stream)
        for _ in range(10):
            sem.vec_axpy(0.5, src, dst)
        c1.record(stream)
        torch.cuda.synchronize()
        stream_gbs = 3 * src.numel() * 8 / (c0.elapsed_time(c1) / 1e3 / 10) / 1e9
        del src, dst

        # ---- generic compressed-row gather-scatter (sem_gs) over this box's
        # global ids g = I + (nx N + 1)(J + (ny N + 1) K), built on the host
        ee = np.arange(nx * ny * nz)
        ll = np.arange(N + 1)
        gI = ((ee % nx) * N)[:, None, None, None] + ll[None, None, None, :]
        gJ = (((ee // nx) % ny) * N)[:, None, None, None] + ll[None, None, :, None]
        gK = ((ee // (nx * ny)) * N)[:, None, None, None] + ll[None, :, None, None]
        gid = (gI + (nx * N + 1) * (gJ + (ny * N + 1) * gK)).reshape(-1)
        del gI, gJ, gK
        g_off, g_ids = sem.gs_csr_build(gid)
        del gid
        g_rows, g_copies = g_off.numel() - 1, g_ids.numel()
        g_off, g_ids = g_off.to(dev), g_ids.to(dev)
        wg = w.clone()
        sem.gs(g_off, g_ids, wg)
        c0.record(stream)
        for _ in range(args.ax_reps):
            sem.gs(g_off, g_ids, wg, check=False)
        c1.record(stream)
        torch.cuda.synchronize()
        gs_s = c0.elapsed_time(c1) / 1e3 / args.ax_reps
        # algorithmic bytes: each copy read and written (16 B) plus its id (4 B); offsets (4 B/row)
        gs_bytes = 20.0 * g_copies + 4.0 * (g_rows + 1)
        gs_info = {"rows": g_rows, "copies": g_copies, "us": gs_s * 1e6,
                   "algorithmic_bytes": gs_bytes, "gbs": gs_bytes / gs_s / 1e9}
        print(f"[bench] gs_csr: {gs_info}", file=sys.stderr, flush=True)
        del g_off, g_ids, wg

        # ---- precision form: inner-outer CG with the FP32 / BF16 operator
        mixed = {}
        x64 = x.clone()
        c_w = A.export(sem._lib.SEM_FIELD_C)
        variants = () if args.skip_mixed else (("f32", False), ("f32", True), ("bf16", False), ("bf16", True))
        for prec, mf in variants:
            key = prec + ("_mfma" if mf else "")
            Am = sem.SemOperator(nx, ny, nz, N, amp, lowprec=prec, device=dev, mfma=mf)
            # the low-precision element operator alone (one launch, FP32 in/out)
            u32 = u.to(torch.float32)
            w32 = torch.empty_like(u32)
            for _ in range(3):
                Am.ax_lowp(u32, sem.LOCAL, out=w32)
            l0 = torch.cuda.Event(enable_timing=True)
            l1 = torch.cuda.Event(enable_timing=True)
            l0.record(stream)
            for _ in range(args.ax_reps):
                Am.ax_lowp(u32, sem.LOCAL, out=w32)
            l1.record(stream)
            torch.cuda.synchronize()
            lowp_ax_us = l0.elapsed_time(l1) * 1e3 / args.ax_reps
            del u32, w32
            xm = torch.empty_like(b)
            for _ in range(max(1, args.warmup)):
                Am.cg(b, xm, rtol=rtol, mixed=True)
            torch.cuda.synchronize()
            msteps = max(1, args.steps // 2)
            t0m = time.perf_counter()
            inner = outer = 0
            for _ in range(msteps):
                _, rm = Am.cg(b, xm, rtol=rtol, mixed=True)
                inner += rm.iters
                outer += rm.outer_iters
            torch.cuda.synchronize()
            wm = time.perf_counter() - t0m
            err = math.sqrt(float((c_w * (xm - x64) ** 2).sum()) / float((c_w * x64 ** 2).sum()))
            mixed[key] = {
                "contractions": "mfma" if mf else "valu",
                "ax_local_us": lowp_ax_us,
                "ax_local_gdofs": A.E * N ** 3 / lowp_ax_us / 1e3,
                "solves_per_s": msteps / wm,
                "ms_per_solve": wm / msteps * 1e3,
                "inner_iters_per_solve": inner / msteps,
                "outer_iters_per_solve": outer / msteps,
                "rel_res_fp64": rm.rel_res,
                "rel_err_vs_fp64_solution": err,
                "status": rm.status,
            }
            print(f"[bench] mixed {key}: {mixed[key]}", file=sys.stderr, flush=True)
            del Am, xm
        torch.cuda.synchronize()

    ax_study = None if args.skip_ax_study else bench_ax_study(args, dev)
    c1 = None if args.skip_c1 else bench_c1(args, dev)
    precision_n11 = None if args.skip_n11 else bench_precision_order(args, dev, 11)
    tuned = None
    if not args.skip_tune:
        from paper_2606_12650_amd import autotune

        t0 = time.perf_counter()
        tuned = autotune.tune_solver(orders=(7, 11), device=dev, cache_path=None)
        print(f"[bench] kernel-shape search ({time.perf_counter() - t0:.1f} s): "
              + "; ".join(f"{p} N={n}: op {r['op_tile']} update {r['update_tile']}"
                          for p, d in tuned.items() for n, r in d.items()), file=sys.stderr, flush=True)
    batching = None if args.skip_batch else bench_batching(args, dev)
    serving = None if args.skip_serve else bench_serving(args, dev)

    E, L = A.E, A.L
    gdof = E * N ** 3
    value = gdof * timed_iters / wall / 1e9
    ax_bytes = 64.0 * L  # read u (1) + G (6), write w (1) doubles per node
    achieved = ax_bytes / ax_s / 1e9
    khash = _kernel_source_hash()
    traffic = _traffic_from_profile(khash)
    s_frac = 1.0 - ((N - 1) / (N + 1)) ** 3
    cg_bytes_per_iter = (19 + 2 * s_frac) * 8.0 * L
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: continuous uniform[-1,1] RHS per global node (seed 4), homogeneous Dirichlet",
        "config": {
            "workload": "Jacobi-PCG to 1e-8 rel. residual, 32x32x32 hex box, N=7, "
                        "deformed x+=0.05 sin(2pi x)sin(2pi y)sin(2pi z)",
            "E": E, "N": N, "L": L, "gdof_per_iter": gdof, "rtol": rtol,
        },
        "solves_per_s": args.steps / wall,
        "mixed": {k: dict(v, speedup_vs_fp64=v["solves_per_s"] / (args.steps / wall)) for k, v in mixed.items()},
        "cg_iters_per_solve": timed_iters / args.steps,
        "cg_event_ms_per_step": ev_ms / args.steps,
        # the unfused (19 + 2s)-word floor per point and iteration over the
        # time, against the peak: a throughput on a fixed byte count, not the
        # bytes this design moves (17 words; see cg_hbm_traffic_frac)
        "cg_unfused_floor_bytes_frac": cg_bytes_per_iter * timed_iters / wall / 1e9 / HBM_PEAK_GBS,
        "cg_hbm_traffic_frac": _cg_traffic_frac(timed_iters, wall),
        "ax_local_us": ax_s * 1e6,
        "ax_masked_us": axm_s * 1e6,
        "ax_gdofs": gdof / ax_s / 1e9,
        "copy_gbs_measured": copy_gbs,
        "ax_frac_of_measured_copy": achieved / copy_gbs,
        "stream_gbs_measured": stream_gbs,
        "ax_frac_of_measured_stream": achieved / stream_gbs,
        "ax_masked_gdofs": gdof / axm_s / 1e9,
        "gs_csr": gs_info,
        "roofline": {
            "kernel": "ax_mfma_local_kernel<8, PrecF64> (sem_ax element operator, N=7: the "
                      "matrix-core tile, the library default at this order)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": ax_bytes,
            "avg_launch_us": ax_s * 1e6,
            "min_run_avg_launch_us": ax_s_min * 1e6,
            "launches_timed": 5 * args.ax_reps,
            "kernel_source_hash": khash,
            # the D contractions on the matrix cores (f64 MFMA), from the
            # committed counter run: not the bound, reported beside it
            "mfma": _mfma_from_profile(khash, "ax_mfma_local_kernel<8, semk::PrecF64>"),
        },
    }
    if ax_study is not None:
        out["ax_study"] = ax_study
    if c1 is not None:
        out["c1"] = c1
    if precision_n11 is not None:
        out["precision_n11"] = precision_n11
    if tuned is not None:
        # per (family, order): microseconds per CG iteration of every candidate
        # element tile (1 matrix-core, 2 vector-ALU) and update tile shape
        # (0 the default), and the chosen ones
        out["autotune_solver"] = tuned
    if batching is not None:
        out["batching"] = batching
    if serving is not None:
        out["serving"] = serving
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(int(round(timed_iters / args.steps)))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
