"""Summaries of rocprofv3 output for the kernels of this library.

``kernel-stats``: per-kernel call count and average duration from a
rocprofv3 ``--kernel-trace --stats`` run (its ``*_results.db`` via
``rocpd2summary``, or a ``kernels_summary.csv``).

``counters``: HBM bytes per dispatch from two ``--pmc`` runs (FETCH_SIZE,
then WRITE_SIZE, csv output), each scaled by what the same counter reads for
a plain device copy of known size in the same run (the bench copies 1 GiB),
written as JSON for ``bench.py``'s ``roofline.traffic``.

Usage:
  python -m paper_2606_12650_amd.profiling kernel-stats <kernels_summary.csv> [--top N]
  python -m paper_2606_12650_amd.profiling counters <fetch_counter_collection.csv>
      <write_counter_collection.csv> <kernel substring> <algorithmic bytes> <source hash>
"""

from __future__ import annotations

import argparse
import csv
import json
import sys
from collections import defaultdict

COPY_BYTES = 1 << 30  # the bench's plain copy: 2^27 doubles


def kernel_stats(path: str, top: int = 15) -> str:
    rows = list(csv.DictReader(open(path)))
    lines = ["| kernel | calls | average (us) | total (ms) | share |", "|---|---|---|---|---|"]
    for r in rows[:top]:
        lines.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['Average (Nsec)']) / 1e3:.1f} | "
                     f"{float(r['Duration (Nsec)']) / 1e6:.1f} | {float(r['Percent (Inc)']):.1f}% |")
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


def counters(fetch_csv: str, write_csv: str, kernel: str, algo_bytes: float, src_hash: str) -> dict:
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
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "copy_bytes": COPY_BYTES,
        "hbm_bytes_per_launch": main["hbm_bytes"],
        "algorithmic_bytes_per_launch": algo_bytes,
        "traffic_over_algorithmic": main["hbm_bytes"] / algo_bytes,
        "all_kernels": summary,
    }


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
    args = ap.parse_args(argv)
    if args.cmd == "kernel-stats":
        print(kernel_stats(args.csv, args.top))
    else:
        print(json.dumps(counters(args.fetch_csv, args.write_csv, args.kernel, args.algo_bytes,
                                  args.src_hash), indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
