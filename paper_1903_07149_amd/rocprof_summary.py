"""Condenses rocprofv3 CSV output into a short markdown summary.

  python -m paper_1903_07149_amd.rocprof_summary stats <prefix>_kernel_stats.csv "<command>"
  python -m paper_1903_07149_amd.rocprof_summary counters <counter_collection.csv> "<command>"

`stats` lists per-kernel call counts and durations; `counters` lists, per
kernel, the mean per-dispatch value of every collected counter.
"""
from __future__ import annotations

import csv
import re
import sys
from collections import defaultdict


def _short(name: str) -> str:
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    name = re.sub(r"HIP_vector_type<float, 4u>", "float4", name)
    return name


def stats(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"command: `{command}`", "",
           "| kernel | calls | avg us | min us | max us | % time |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def counters(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    acc = defaultdict(lambda: defaultdict(list))
    for r in rows:
        name = r.get("Kernel_Name") or r.get("Kernel-Name") or ""
        cname = r.get("Counter_Name") or r.get("Counter-Name")
        val = r.get("Counter_Value") or r.get("Counter-Value")
        disp = r.get("Dispatch_Id") or r.get("Dispatch-Id")
        if cname is None or val is None:
            continue
        acc[_short(name)][cname].append((disp, float(val)))
    out = [f"command: `{command}`", "", "| kernel | counter | dispatches | mean per dispatch |",
           "|---|---|---:|---:|"]
    for k, cs in acc.items():
        for c, vals in cs.items():
            per = defaultdict(float)
            for d, v in vals:
                per[d] += v
            m = sum(per.values()) / max(1, len(per))
            out.append(f"| `{k}` | {c} | {len(per)} | {m:.1f} |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    kind, path, cmd = sys.argv[1], sys.argv[2], sys.argv[3]
    sys.stdout.write(stats(path, cmd) if kind == "stats" else counters(path, cmd))
