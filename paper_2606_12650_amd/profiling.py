"""Summaries of rocprofv3 output for the kernels of this library.

``kernel-stats``: per-kernel call count and average duration from a
rocprofv3 ``--kernel-trace --stats`` run (its ``*_results.db`` via
``rocpd2summary``, or a ``kernels_summary.csv``).

``counters``: HBM bytes per dispatch from two ``--pmc`` runs (FETCH_SIZE,
then WRITE_SIZE, csv output), each scaled by what the same counter reads for
a plain device copy of known size in the same run (the bench copies 1 GiB),
written as JSON for ``bench.py``'s ``roofline.traffic``.

``mfma``: matrix-core use per kernel from one ``--pmc`` run of
SQ_INSTS_VALU_MFMA_MOPS_{F64,F32,BF16} (units of 512 flops),
SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE, with the kernels' average
durations from a ``--kernel-trace --stats`` summary of the same command:
MFMA flops per dispatch, achieved MFMA FLOP/s against the dense peak of the
instruction's type, and the busy fraction
SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE per XCD * 256 CUs * 4 SIMDs).
rocprofv3 sums GRBM_GUI_ACTIVE over the 8 XCDs in its csv (it reads about
8 x 2.4 GHz x the kernel time); the cycles of one XCD are that sum / 8.

Usage:
  python -m paper_2606_12650_amd.profiling kernel-stats <kernels_summary.csv> [--top N]
  python -m paper_2606_12650_amd.profiling counters <fetch_counter_collection.csv>
      <write_counter_collection.csv> <kernel substring> <algorithmic bytes> <source hash>
      [--cg-hash <hash of the CG kernels' sources>]
  python -m paper_2606_12650_amd.profiling mfma <counter_collection.csv> <kernels_summary.csv>
      <source hash> <kernel substring> [<kernel substring> ...]
"""

from __future__ import annotations

import argparse
import csv
import json
import sys
from collections import defaultdict

COPY_BYTES = 1 << 30  # the bench's plain copy: 2^27 doubles


def _stats_rows(path: str) -> list[dict]:
    """Rows of a kernel summary: rocpd2summary's kernels_summary.csv or
    rocprofv3's own *_kernel_stats.csv (--stats with csv output), as
    (name, calls, average ns, total ns, percent) dicts sorted by total."""
    out = []
    for r in csv.DictReader(open(path)):
        if "Average (Nsec)" in r:
            out.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_ns": float(r["Average (Nsec)"]),
                        "total_ns": float(r["Duration (Nsec)"]), "pct": float(r["Percent (Inc)"])})
        else:
            out.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                        "total_ns": float(r["TotalDurationNs"]), "pct": float(r["Percentage"])})
    out.sort(key=lambda r: -r["total_ns"])
    return out


def kernel_stats(path: str, top: int = 15) -> str:
    lines = ["| kernel | calls | average (us) | total (ms) | share |", "|---|---|---|---|---|"]
    for r in _stats_rows(path)[:top]:
        name = r["name"].replace("semk::(anonymous namespace)::", "")
        lines.append(f"| `{name[:110]}` | {r['calls']} | {r['avg_ns'] / 1e3:.1f} | "
                     f"{r['total_ns'] / 1e6:.1f} | {r['pct']:.1f}% |")
    return "\n".join(lines)


def _per_kernel(path: str):
    rows = list(csv.DictReader(open(path)))
    out = defaultdict(list)
    copies = []
    for r in rows:
        v = float(r["Counter_Value"]) * 1024.0  # KiB per dispatch -> bytes
        out[r["Kernel_Name"]].append(v)
        if "copyBuffer" in r["Kernel_Name"]:
            copies.append(v)
    return out, copies


def counters(fetch_csv: str, write_csv: str, kernel: str, algo_bytes: float, src_hash: str,
             cg_hash: str | None = None) -> dict:
    fetch, fcopies = _per_kernel(fetch_csv)
    write, wcopies = _per_kernel(write_csv)
    # the copy of known size: the largest copy dispatches read and write 1 GiB
    f_copy = max(fcopies)
    w_copy = max(wcopies)
    f_scale = COPY_BYTES / f_copy
    w_scale = COPY_BYTES / w_copy
    summary = {}
    for name in fetch:
        fv = [v for v in fetch[name] if v > 0]
        wv = [v for v in write.get(name, []) if v > 0]
        if not fv:
            continue
        f = max(fv)  # dispatches that skipped (converged solves) read ~0
        w = max(wv) if wv else 0.0
        summary[name] = {"fetch_bytes": f * f_scale, "write_bytes": w * w_scale,
                         "hbm_bytes": f * f_scale + w * w_scale, "dispatches": len(fetch[name])}
    match = [n for n in summary if kernel in n]
    if not match:
        raise SystemExit(f"kernel {kernel!r} not in the counter runs")
    main = summary[match[0]]
    return {
        "kernel": match[0],
        "kernel_source_hash": src_hash,
        "cg_source_hash": cg_hash,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "copy_bytes": COPY_BYTES,
        "hbm_bytes_per_launch": main["hbm_bytes"],
        "algorithmic_bytes_per_launch": algo_bytes,
        "traffic_over_algorithmic": main["hbm_bytes"] / algo_bytes,
        "all_kernels": summary,
    }


# Dense matrix-core peaks of MI355X (AMD published, no sparsity), TFLOP/s.
MFMA_PEAK_TFLOPS = {"F64": 78.6, "F32": 157.3, "BF16": 2500.0}
MOPS_FLOPS = 512.0
N_CU, SIMD_PER_CU, N_XCD = 256, 4, 8


def _counters_by_dispatch(path: str):
    """{kernel: [{counter: value} per dispatch]} from a multi-counter csv."""
    per = defaultdict(dict)
    names = {}
    for r in csv.DictReader(open(path)):
        did = r.get("Dispatch_Id") or r.get("Correlation_Id") or str(len(per))
        names[did] = r["Kernel_Name"]
        per[did][r["Counter_Name"]] = per[did].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    out = defaultdict(list)
    for did, vals in per.items():
        out[names[did]].append(vals)
    return out


def mfma(pmc_csv: str, stats_csv: str, src_hash: str, kernels: list[str]) -> dict:
    disp = _counters_by_dispatch(pmc_csv)
    durs = {r["name"]: r["avg_ns"] for r in _stats_rows(stats_csv)}
    res = {}
    for sub in kernels:
        names = [n for n in disp if sub in n]
        if not names:
            raise SystemExit(f"kernel {sub!r} not in the counter run")
        name = names[0]
        ds = disp[name]
        dur = next((v for k, v in durs.items() if sub in k), None)
        # dispatches that did work (a converged solve's launches return at once)
        busy = [d for d in ds if sum(d.get(f"SQ_INSTS_VALU_MFMA_MOPS_{t}", 0.0) for t in MFMA_PEAK_TFLOPS) > 0]
        if not busy:
            res[sub] = {"kernel": name, "dispatches": len(ds), "mfma_flops_per_dispatch": 0.0}
            continue
        row = {"kernel": name, "dispatches": len(ds), "dispatches_with_mfma": len(busy)}
        flops = {}
        for t in MFMA_PEAK_TFLOPS:
            v = max(d.get(f"SQ_INSTS_VALU_MFMA_MOPS_{t}", 0.0) for d in busy) * MOPS_FLOPS
            if v > 0:
                flops[t] = v
        dtype = max(flops, key=flops.get)
        row["mfma_flops_per_dispatch"] = flops
        row["dtype"] = dtype
        b = max(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in busy)
        g = max(d.get("GRBM_GUI_ACTIVE", 0.0) for d in busy)
        row["busy_cycles"] = b
        row["gui_active_cycles_per_xcd"] = g / N_XCD
        row["busy_frac"] = b / (g / N_XCD * N_CU * SIMD_PER_CU) if g > 0 else None
        if dur:
            row["avg_us"] = dur / 1e3
            row["clock_ghz_check"] = g / N_XCD / dur
            ach = flops[dtype] / (dur * 1e-9) / 1e12
            row["achieved_tflops"] = ach
            row["peak_tflops"] = MFMA_PEAK_TFLOPS[dtype]
            row["util"] = ach / MFMA_PEAK_TFLOPS[dtype]
        res[sub] = row
    return {"kernel_source_hash": src_hash, "kernels": res}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("kernel-stats")
    a.add_argument("csv")
    a.add_argument("--top", type=int, default=15)
    b = sub.add_parser("counters")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("kernel")
    b.add_argument("algo_bytes", type=float)
    b.add_argument("src_hash")
    b.add_argument("--cg-hash", default=None, help="source hash of the CG iteration's kernels")
    m = sub.add_parser("mfma")
    m.add_argument("pmc_csv")
    m.add_argument("stats_csv")
    m.add_argument("src_hash")
    m.add_argument("kernels", nargs="+")
    args = ap.parse_args(argv)
    if args.cmd == "kernel-stats":
        print(kernel_stats(args.csv, args.top))
    elif args.cmd == "mfma":
        print(json.dumps(mfma(args.pmc_csv, args.stats_csv, args.src_hash, args.kernels), indent=1))
    else:
        print(json.dumps(counters(args.fetch_csv, args.write_csv, args.kernel, args.algo_bytes,
                                  args.src_hash, args.cg_hash), indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
