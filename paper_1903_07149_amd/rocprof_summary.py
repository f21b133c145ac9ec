"""Condenses rocprofv3 CSV output into a short markdown summary.

  python -m paper_1903_07149_amd.rocprof_summary stats <prefix>_kernel_stats.csv "<command>"
  python -m paper_1903_07149_amd.rocprof_summary counters <counter_collection.csv> "<command>"
  python -m paper_1903_07149_amd.rocprof_summary traffic <fetch.csv> <write.csv> <kernel>
         <algorithmic bytes per launch> <source digest> <workload> "<fetch cmd>" "<write cmd>"

`stats` lists per-kernel call counts and durations; `counters` lists, per
kernel, the mean per-dispatch value of every collected counter; `traffic`
turns one FETCH_SIZE and one WRITE_SIZE run (KiB per dispatch) into HBM bytes
per launch of <kernel>, each counter scaled by what it reads for the
512 MiB device copy (`__amd_rocclr_copyBuffer`) of the same run, and prints
the JSON record the benchmark reads.
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


def _per_dispatch(path: str, counter: str) -> dict:
    """kernel name -> list of per-dispatch sums of one counter."""
    per = defaultdict(lambda: defaultdict(float))
    for r in csv.DictReader(open(path)):
        cname = r.get("Counter_Name") or r.get("Counter-Name")
        if cname != counter:
            continue
        name = _short(r.get("Kernel_Name") or r.get("Kernel-Name") or "")
        disp = r.get("Dispatch_Id") or r.get("Dispatch-Id")
        per[name][disp] += float(r.get("Counter_Value") or r.get("Counter-Value"))
    return {k: list(v.values()) for k, v in per.items()}


COPY_BYTES = 512 << 20
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def traffic(fetch_csv: str, write_csv: str, kernel: str, algorithmic: int, digest: str,
            workload: str, fetch_cmd: str, write_cmd: str) -> dict:
    f = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _per_dispatch(write_csv, "WRITE_SIZE")

    def pick(d, key):
        hits = [v for k, v in d.items() if key in k]
        if not hits:
            raise SystemExit(f"no dispatch of {key} in the counter output")
        return hits[0]

    def copy_kib(d):
        # the calibration copy is the largest copyBuffer dispatch of the run
        return max(pick(d, COPY_KERNEL))

    fk, wk = pick(f, kernel), pick(w, kernel)
    f_mean, w_mean = sum(fk) / len(fk), sum(wk) / len(wk)
    f_fac = COPY_BYTES / 1024 / copy_kib(f)
    w_fac = COPY_BYTES / 1024 / copy_kib(w)
    rd = f_mean * 1024 * f_fac
    wr = w_mean * 1024 * w_fac
    return {"kernel": kernel, "workload": workload,
            "fetch_size_kib_per_dispatch": round(f_mean, 1),
            "write_size_kib_per_dispatch": round(w_mean, 1),
            "dispatches": [len(fk), len(wk)],
            "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib_read": round(copy_kib(f), 1),
                                 "write_kib_read": round(copy_kib(w), 1),
                                 "fetch_factor": round(f_fac, 4), "write_factor": round(w_fac, 4)},
            "read_bytes_per_launch": int(rd), "write_bytes_per_launch": int(wr),
            "bytes_per_launch": int(rd + wr), "algorithmic_bytes_per_launch": int(algorithmic),
            "kernel_source_sha256_16": digest, "commands": [fetch_cmd, write_cmd]}


if __name__ == "__main__":
    kind = sys.argv[1]
    if kind == "traffic":
        import json
        a = sys.argv[2:]
        print(json.dumps(traffic(a[0], a[1], a[2], int(a[3]), a[4], a[5], a[6], a[7]), indent=1))
    else:
        path, cmd = sys.argv[2], sys.argv[3]
        sys.stdout.write(stats(path, cmd) if kind == "stats" else counters(path, cmd))
