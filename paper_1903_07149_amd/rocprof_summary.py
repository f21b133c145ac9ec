"""Condenses rocprofv3 CSV output into a short markdown summary.

  python -m paper_1903_07149_amd.rocprof_summary stats <prefix>_kernel_stats.csv "<command>"
  python -m paper_1903_07149_amd.rocprof_summary counters <counter_collection.csv> "<command>"
  python -m paper_1903_07149_amd.rocprof_summary traffic <fetch.csv> <write.csv> <kernel>
         <algorithmic bytes per launch> <source digest> <workload> "<fetch cmd>" "<write cmd>"
  python -m paper_1903_07149_amd.rocprof_summary derived <sq1.csv> <sq2.csv> <fetch.csv>
         <write.csv> <kernel substring>[,<kernel substring>...] [first=N] [grid=G]
         (separate the substrings with ';' instead when they contain commas)

`stats` lists per-kernel call counts and durations; `counters` lists, per
kernel, the mean per-dispatch value of every collected counter; `traffic`
turns one FETCH_SIZE and one WRITE_SIZE run (KiB per dispatch) into HBM bytes
per launch of <kernel>, each counter scaled by what it reads for the
512 MiB device copy (`__amd_rocclr_copyBuffer`) of the same run, and prints
the JSON record the benchmark reads.  `derived` turns two SQ counter passes
(instruction counts, then wait cycles) and one FETCH_SIZE and one WRITE_SIZE
pass into per-kernel rates: VALU wave instructions per CU-clock (the issue
ceiling is one), VALU lane utilisation, LDS instructions and LDS-busy cycles
per CU-clock, the share of wave cycles spent waiting, and calibrated HBM
bytes per dispatch (optionally only the first N dispatches, or only the
dispatches of grid size G).
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


def _per_dispatch_all(path: str, grid: int | None = None) -> dict:
    """kernel -> counter -> {dispatch: value} (values of one dispatch summed)."""
    per = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))
    for r in csv.DictReader(open(path)):
        cname = r.get("Counter_Name") or r.get("Counter-Name")
        if cname is None:
            continue
        if grid is not None and int(r.get("Grid_Size") or r.get("Grid-Size") or 0) != grid:
            continue
        name = _short(r.get("Kernel_Name") or r.get("Kernel-Name") or "")
        disp = int(r.get("Dispatch_Id") or r.get("Dispatch-Id"))
        per[name][cname][disp] += float(r.get("Counter_Value") or r.get("Counter-Value"))
    return per


def derived(paths: list[str], kernels: list[str], first: int | None = None,
            grid: int | None = None) -> tuple[str, dict]:
    """Mean per-dispatch counters of each kernel matching one of `kernels` and
    the rates derived from them (see the module docstring)."""
    merged = defaultdict(dict)
    copy = {}
    for path in paths:
        for name, cs in _per_dispatch_all(path).items():
            if COPY_KERNEL in name:
                for c, d in cs.items():
                    copy[c] = max(d.values())
        for name, cs in _per_dispatch_all(path, grid).items():
            key = next((k for k in kernels if k in name), None)
            if key is None:
                continue
            for c, d in cs.items():
                vals = [d[i] for i in sorted(d)]
                if first:
                    vals = vals[:first]
                merged[key][c] = (sum(vals) / len(vals), len(vals))
    rows = ["| kernel | dispatches | us (GRBM) | VALU instr | VALU / CU-clk | lane util | "
            "LDS instr | LDS busy / CU-clk | wait / wave-cycles | VMEM instr | HBM read MB | "
            "HBM write MB |", "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    out = {}
    for k in kernels:
        cs = merged.get(k)
        if not cs:
            continue
        g = lambda c: cs[c][0] if c in cs else float("nan")
        cyc = g("GRBM_GUI_ACTIVE") / 8          # summed over the 8 XCDs
        rd = g("FETCH_SIZE") * 1024 * (COPY_BYTES / 1024 / copy["FETCH_SIZE"]) \
            if "FETCH_SIZE" in cs and "FETCH_SIZE" in copy else float("nan")
        wr = g("WRITE_SIZE") * 1024 * (COPY_BYTES / 1024 / copy["WRITE_SIZE"]) \
            if "WRITE_SIZE" in cs and "WRITE_SIZE" in copy else float("nan")
        d = {"dispatches": cs.get("SQ_INSTS_VALU", (0, 0))[1],
             "us": cyc / 2400.0,
             "valu_insts": g("SQ_INSTS_VALU"),
             "valu_per_cu_clk": g("SQ_INSTS_VALU") / 256 / cyc,
             "lane_util": g("SQ_THREAD_CYCLES_VALU") / 64 / g("SQ_ACTIVE_INST_VALU"),
             "lds_insts": g("SQ_INSTS_LDS"),
             "lds_busy_per_cu_clk": g("SQ_LDS_IDX_ACTIVE") / 256 / cyc,
             "wait_frac": g("SQ_WAIT_ANY") / g("SQ_WAVE_CYCLES"),
             "wait_inst_frac": g("SQ_WAIT_INST_ANY") / g("SQ_WAVE_CYCLES"),
             "lds_wait_frac": g("SQ_WAIT_INST_LDS") / g("SQ_WAVE_CYCLES"),
             "vmem_insts": g("SQ_INSTS_VMEM"),
             "hbm_read_bytes": rd, "hbm_write_bytes": wr}
        out[k] = d
        rows.append(f"| `{k}` | {d['dispatches']} | {d['us']:.1f} | {d['valu_insts']:.3e} | "
                    f"{d['valu_per_cu_clk']:.3f} | {d['lane_util']:.3f} | {d['lds_insts']:.3e} | "
                    f"{d['lds_busy_per_cu_clk']:.3f} | {d['wait_frac']:.3f} | "
                    f"{d['vmem_insts']:.3e} | {rd / 1e6:.2f} | {wr / 1e6:.2f} |")
    return "\n".join(rows) + "\n", out


if __name__ == "__main__":
    kind = sys.argv[1]
    if kind == "derived":
        a = sys.argv[2:]
        opts = dict(x.split("=", 1) for x in a[5:])
        names = a[4].split(";") if ";" in a[4] else a[4].split(",")
        sys.stdout.write(derived(a[:4], names, int(opts["first"]) if "first" in opts
                                 else None, int(opts["grid"]) if "grid" in opts else None)[0])
    elif kind == "traffic":
        import json
        a = sys.argv[2:]
        print(json.dumps(traffic(a[0], a[1], a[2], int(a[3]), a[4], a[5], a[6], a[7]), indent=1))
    else:
        path, cmd = sys.argv[2], sys.argv[3]
        sys.stdout.write(stats(path, cmd) if kind == "stats" else counters(path, cmd))
