#!/usr/bin/env python3
"""Throughput of the SCALP clustering path on one MI355X.

Headline: Mpixel-iterations/s of hard SCALP on the 1920x1080 synthetic
Voronoi workload with k = 2000 and 10 iterations.  One step is one whole job
from inputs resident in HBM: pack (l, a, b, w) and grid initialisation
(eager), then 10 x (fused assignment + update, finalize + Eq. (4)
projection) as one hipGraph replay.

Also reported on the same JSON line:
  roofline      the fused assignment kernel (the dominant kernel): the method's
                algorithmic FP32 operations per launch / its average duration,
                measured with HIP events around every launch in a second loop
                of the same steps launched kernel by kernel
                (eager_ms_per_step), against the published FP32 peak; beside
                it, under "binding", what the kernel executes against the
                resource that binds it (VALU issue, from the committed SQ
                counter record while the kernel source matches it);
  without_pruning  the same step with every candidate's path walked
                (exact_pruning = 0, same labels): its rate, the kernel's
                average launch time and that roofline fraction;
  cpu_baseline  the plain C oracle timed on this host's cores on the same
                workload;
  extensions    the ragged 64-image batch in one persistent launch per
                iteration (hipGraph), against the same images run one by one
                through the single-image path, and soft SCALP forward+backward.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel-iter/s (assign+update) 1080p K=2000; batched and soft fwd+bwd MP/s"

# MI355X published peaks.  FP32 vector: 157.3 TFLOP/s (256 CUs x 2.4 GHz x
# 256 FLOP per CU-clock, i.e. 4 SIMDs x 16 lanes issuing a packed FMA that
# counts as 4 operations); HBM3E: 8 TB/s.
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBPS = 8000.0
# VALU issue ceiling derived from the unit counts: each of a CU's 4 SIMDs
# retires a wave64 VALU instruction every 4 clocks, so one wave64 instruction
# per CU-clock, 256 x 2.4e9 = 614.4 G instructions/s (39.3 T lane-ops/s).
# Integer-heavy streams were measured slightly above it (1.19 per CU-clock,
# profiles/peaks_mi355x.md), so it is a ceiling for FP32 work.
VALU_ISSUE_PEAK_GINSTS = 256 * 2.4
# LDS: 256 B per CU-clock on CDNA4 = 157.3 TB/s spec; the conflict-free
# ds_read_b128 rate measured by peaks_probe is 107.5 TB/s.
LDS_SPEC_TBPS = 256 * 256 * 2.4e9 / 1e12
LDS_MEASURED_TBPS = 107.5

EXTENSIONS = ("batched", "soft", "window_form", "multiscale", "contour_prior", "quality")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "assign_hd_traffic.json")
ISSUE_FILE = os.path.join(ROOT, "profiles", "assign_hd_sq.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1903_07149_amd", "csrc", f)
                  for f in ("scalp_kernels.hip", "scalp_device.h")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_digest() -> str:
    """Fingerprint of the assignment kernel's sources (the traffic figures taken
    with hardware counters are only reported while it matches)."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extensions", action="store_true")
    ap.add_argument("--extensions", default=None,
                    help="comma-separated subset of: batched, soft, window_form, "
                         "multiscale, contour_prior, quality (default: all)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 512 MiB device copy (counter calibration)")
    ap.add_argument("--launch", default=None,
                    help="WG,LDS_PIXELS[,TABLE_MODE]: fixed assignment launch shape instead of "
                         "autotuning")
    ap.add_argument("--batch-launch", default=None,
                    help="WG,LDS_PIXELS,BLOCKS_PER_CU[,TABLE_MODE]: fixed launch shape of the "
                         "batched persistent kernel instead of autotuning it on the batch")
    return ap.parse_args()


def batch_launch(text: str) -> dict:
    """--batch-launch WG,LDS_PIXELS,BLOCKS_PER_CU[,TABLE_MODE] as launch keywords."""
    v = [int(x) for x in text.split(",")]
    out = {"wg_size": v[0], "lds_pixels": v[1], "persistent_blocks": v[2]}
    if len(v) > 3:
        out["table_mode"] = v[3]
    return out


def traffic_for(digest: str):
    """HBM bytes per launch of the assignment kernel from the committed counter
    summary, if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != digest:
        return None
    return t.get("bytes_per_launch")


def issue_for(digest: str):
    """VALU and LDS wave instructions per launch of the assignment kernel
    from the committed SQ counter record, if it was taken on the current
    kernel source."""
    try:
        with open(ISSUE_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != digest:
        return None
    return t


def binding_resource(issue, launch_s):
    """What the fused assignment kernel actually executes, against the resource
    that binds it (VALU issue): wave64 VALU instructions per launch from the
    committed SQ counter record over the launch time measured in this run,
    against one instruction per CU-clock; LDS bytes from the LDS instruction
    count (8 bytes per lane: table reads and writes, bin atomics) against the
    measured ds_read ceiling.  Marked stale, with no fractions, when the
    record was taken on other kernel sources."""
    if issue is None:
        return {"resource": "VALU issue", "stale": True, "frac": None,
                "note": "no SQ counter record for the current kernel sources"}
    insts = issue["valu_insts_per_dispatch"]
    g_insts = insts / launch_s / 1e9
    lds_b = 64 * 8 * issue["lds_insts_per_dispatch"]
    return {"resource": "VALU issue", "stale": False,
            "valu_insts_per_launch": int(insts),
            "achieved": round(g_insts, 1), "peak": VALU_ISSUE_PEAK_GINSTS,
            "unit": "G wave64 VALU instructions/s",
            "frac": round(g_insts / VALU_ISSUE_PEAK_GINSTS, 4),
            "lds_bytes_per_launch": int(lds_b),
            "lds_TBps": round(lds_b / launch_s / 1e12, 2),
            "lds_frac_of_measured": round(lds_b / launch_s / 1e12 / LDS_MEASURED_TBPS, 4),
            "counter_record": os.path.relpath(ISSUE_FILE, ROOT)}


def alu_roofline(flops: float, seconds: float, timed: str) -> dict:
    """Algorithmic FP32 work of one assignment pass over the measured time of
    one iteration (`timed` says what that time includes: with the update and
    projection kernels in it, the rate is a lower bound on the assignment
    kernel's), against the published FP32 peak."""
    a = flops / seconds / 1e12
    return {"bound": "alu", "achieved": round(a, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(a / FP32_PEAK_TFLOPS, 4), "flops_per_iteration": int(flops),
            "timed": timed}


def bench_hard(torch, args):
    from paper_1903_07149_amd import autotune, counts, synth
    from paper_1903_07149_amd.scalp import Scalp

    wl = synth.HD
    img = synth.workload_image(wl)
    H, W = img.contour.shape
    lab = torch.from_numpy(img.lab).cuda()
    con = torch.from_numpy(img.contour).cuda()
    if args.launch:
        v = [int(x) for x in args.launch.split(",")]
        tuned = {"wg_size": v[0], "lds_pixels": v[1]}
        if len(v) > 2:
            tuned["table_mode"] = v[2]
        log(f"fixed launch shape: {tuned}")
    else:
        tuned = autotune.tune(W, H, wl.k, lab, con, use_cache=False)
        log(f"autotuned launch shape: {tuned}")
    s = Scalp(W, H, wl.k, iterations=wl.iterations, **tuned)
    c, e, l, n = s.new_state()
    iters = wl.iterations

    def step(evs=None):
        s.init_grid(lab, con, out=(c, e, l))
        for it in range(iters):
            if evs is not None:
                evs[it][0].record()
            s.assign_accumulate(c, e, l)
            if evs is not None:
                evs[it][1].record()
            s.finalize(l, c, e, n)

    # algorithmic work of every iteration (the run is deterministic)
    s.init_grid(lab, con, out=(c, e, l))
    work = []
    for it in range(iters):
        torch.cuda.synchronize()
        work.append(counts.pass_work(W, H, s.grid.nx, s.grid.ny, e.cpu().numpy()))
        s.assign_accumulate(c, e, l)
        s.finalize(l, c, e, n)
    torch.cuda.synchronize()

    # the timed region: the 10 iterations as one hipGraph replay (the
    # iteration driver), each step preceded by the eager pack + grid init
    gr = s.graph(c, e, l, n)
    for _ in range(args.warmup):
        s.init_grid(lab, con, out=(c, e, l))
        gr.launch()
    torch.cuda.synchronize()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    g0.record()
    for _ in range(args.steps):
        s.init_grid(lab, con, out=(c, e, l))
        gr.launch()
    g1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = g0.elapsed_time(g1) / args.steps
    gr.close()

    # the same steps launched one kernel at a time, with HIP events around
    # every assignment launch on the stream it runs on: the kernel's own
    # duration (the events add a little time between launches, so this
    # loop's step time is reported separately, not as the value)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in range(iters)] for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for k in range(args.steps):
        step(evs[k])
    t_end.record()
    torch.cuda.synchronize()
    eager_ms = t_start.elapsed_time(t_end) / args.steps
    per_it = [sum(evs[k][it][0].elapsed_time(evs[k][it][1]) for k in range(args.steps)) / args.steps
              for it in range(iters)]

    # the same step with every candidate's path walked (exact_pruning = 0;
    # the labels are the same): graph replays, then HIP events around each
    # assignment launch
    gr0 = s.graph(c, e, l, n, exact_pruning=0)
    for _ in range(args.warmup):
        s.init_grid(lab, con, out=(c, e, l))
        gr0.launch()
    torch.cuda.synchronize()
    u0 = torch.cuda.Event(enable_timing=True)
    u1 = torch.cuda.Event(enable_timing=True)
    u0.record()
    for _ in range(args.steps):
        s.init_grid(lab, con, out=(c, e, l))
        gr0.launch()
    u1.record()
    torch.cuda.synchronize()
    ms_step0 = u0.elapsed_time(u1) / args.steps
    gr0.close()
    passes0 = 3
    ev0 = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
            for _ in range(iters)] for _ in range(passes0)]
    for q in range(passes0):
        s.init_grid(lab, con, out=(c, e, l))
        for it in range(iters):
            ev0[q][it][0].record()
            s.assign_accumulate(c, e, l, exact_pruning=0)
            ev0[q][it][1].record()
            s.finalize(l, c, e, n, exact_pruning=0)
    torch.cuda.synchronize()
    kern0_s = sum(ev0[q][it][0].elapsed_time(ev0[q][it][1]) for q in range(passes0)
                  for it in range(iters)) / passes0 * 1e-3

    N = W * H
    value = N * iters / (ms_step * 1e-3) / 1e6
    flops = sum(w["flops"] for w in work)
    samples = sum(w["samples"] for w in work)
    kern_s = sum(per_it) * 1e-3
    launch_s = kern_s / iters
    achieved = flops / kern_s / 1e12
    digest = source_digest()
    traffic = traffic_for(digest)
    # achieved: the method's algorithmic FP32 operations (Eqs. (1)-(3) over
    # every candidate's path, counted from the endpoints) per launch over the
    # kernel's measured launch time, against the published FP32 peak
    roofline = {
        "bound": "alu",
        "kernel": (f"k_assign<{s.params.wg_size},true,{'true' if s.params.table_mode else 'false'}> "
                   "(fused assignment + update sums)"),
        "achieved": round(achieved, 3),
        "peak": FP32_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
        "traffic": traffic,
        "avg_launch_ms": round(launch_s * 1e3, 4),
        "flops_per_launch": flops // iters,
        "samples_per_launch": samples // iters,
        "samples_per_px_iter": round(samples / (N * iters), 2),
        "lds_algorithmic_TBps": round(16 * samples / kern_s / 1e12, 3),
        "lds_algorithmic_frac": round(16 * samples / kern_s / 1e12 / LDS_SPEC_TBPS, 4),
        "kernel_source_sha256_16": digest,
    }
    if traffic is not None:
        roofline["hbm_frac"] = round(traffic / launch_s / 1e9 / HBM_PEAK_GBPS, 4)
    roofline["binding"] = binding_resource(issue_for(digest), launch_s)
    without_pruning = {
        "value": round(N * iters / (ms_step0 * 1e-3) / 1e6, 1),
        "ms_per_step": round(ms_step0, 4),
        "avg_launch_ms": round(kern0_s * 1e3 / iters, 4),
        "frac": round(flops / kern0_s / 1e12 / FP32_PEAK_TFLOPS, 4),
    }
    log(f"hard: {ms_step:.3f} ms/step graph, {eager_ms:.3f} ms/step eager with events, "
        f"{ms_step0:.3f} ms/step without pruning, wall {wall:.2f}s")
    if args.copy_probe:
        src = torch.empty(512 * 2**20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 3 x 512 MiB device copies")
    return img, tuned, {
        "value": value, "ms_per_step": ms_step, "eager_ms_per_step": eager_ms,
        "eager_value": N * iters / (eager_ms * 1e-3) / 1e6, "roofline": roofline,
        "without_pruning": without_pruning,
        "config": {"workload": wl.name, "width": W, "height": H, "k": wl.k,
                   "num_sp": s.grid.num_sp, "iterations": iters, "launch": tuned,
                   "step": "pack + grid init (eager) + 10 x (fused assign/update, finalize/projection) "
                           "as one hipGraph replay"},
    }


def cpu_baseline(img, k, iters):
    from oracle import oracle as orc
    orc.lib()
    threads = orc.max_threads()
    H, W = img.contour.shape
    reps = 0
    t0 = time.perf_counter()
    while True:
        orc.run(img.lab, img.contour, k, iterations=iters)
        reps += 1
        el = time.perf_counter() - t0
        # a bounded sample: at least 10 s of CPU work, at most 12 full runs
        if el >= 10.0 or reps >= 12:
            break
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    out = {"value": round(W * H * iters * reps / el / 1e6, 3), "unit": "Mpixel-iter/s",
           "cores": threads, "kind": "oracle", "cpu": cpu, "host_cpus": os.cpu_count(),
           "sample": f"{reps} full run(s) of {W}x{H} k={k}, {iters} iterations, "
                     f"{el:.1f} s on {threads} OpenMP threads"}
    # the same oracle on one thread, over a shorter run of the same workload
    # (the iterations cost about the same, so the rate per pixel-iteration carries over)
    it1 = 2
    orc.set_threads(1)
    try:
        t0 = time.perf_counter()
        orc.run(img.lab, img.contour, k, iterations=it1)
        el1 = time.perf_counter() - t0
    finally:
        orc.set_threads(threads)
    out["one_thread"] = {"value": round(W * H * it1 / el1 / 1e6, 3), "unit": "Mpixel-iter/s",
                         "sample": f"1 run of {W}x{H} k={k}, {it1} iterations, {el1:.1f} s on 1 thread"}
    return out


def bench_batched(torch, args, tuned):
    from paper_1903_07149_amd import counts, synth
    from paper_1903_07149_amd.scalp import Scalp, ScalpBatch

    from paper_1903_07149_amd import autotune
    wls = synth.batch_workloads()
    imgs = [synth.workload_image(w) for w in wls]
    shapes = [(w.width, w.height, w.k) for w in wls]
    lab = torch.cat([torch.from_numpy(i.lab.reshape(-1, 3)) for i in imgs]).cuda()
    con = torch.cat([torch.from_numpy(i.contour.reshape(-1)) for i in imgs]).cuda()
    # launch shape of the persistent kernel, tuned on this batch
    if args.batch_launch:
        tuned_b = batch_launch(args.batch_launch)
    else:
        tuned_b = autotune.tune_batch(shapes, lab, con, use_cache=False)
    log(f"batch launch shape: {tuned_b}")
    b = ScalpBatch(shapes, iterations=10, **tuned_b)
    st = b.new_state()
    gr = b.graph(lab, con, *st)
    for _ in range(2):
        gr.launch()
    torch.cuda.synchronize()
    reps = 5
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        gr.launch()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    gr.close()
    # the same images, one by one, through the single-image path
    singles = []
    for w, i in zip(wls, imgs):
        s = Scalp(w.width, w.height, w.k, iterations=10, **tuned)
        singles.append((s, torch.from_numpy(i.lab).cuda(), torch.from_numpy(i.contour).cuda(),
                        s.new_state()))
    for s, la, co, out in singles:
        s.run(la, co, out=out)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(2):
        for s, la, co, out in singles:
            s.run(la, co, out=out)
    t1.record()
    torch.cuda.synchronize()
    ms1 = t0.elapsed_time(t1) / 2
    px_it = b.total_pixels * 10
    # algorithmic work of one pass at the initial grid of every image
    b0 = ScalpBatch(shapes, iterations=0, **tuned_b)
    _, e0, _, _ = b0.run(lab, con)
    e0 = e0.cpu().numpy()
    flops = 0
    for (s0, s1), g in zip(b0.sp_slices(), b0.grids):
        flops += counts.pass_work(g.width, g.height, g.nx, g.ny, e0[s0:s1])["flops"]
    roof = alu_roofline(flops, ms * 1e-3 / 10,
                        "batched run / 10 (pack, init, then per iteration the persistent "
                        "assignment, finalize and projection); work at the initial grid")
    return {"workload": f"{len(wls)} ragged Voronoi images, H,W in [240,2160], k = HW/1000, 10 it",
            "roofline": roof,
            "launch": tuned_b, "pixels": b.total_pixels, "superpixels": b.total_sp,
            "batched_mpx_iter_s": round(px_it / (ms * 1e-3) / 1e6, 1), "batched_ms": round(ms, 3),
            "single_path_mpx_iter_s": round(px_it / (ms1 * 1e-3) / 1e6, 1),
            "single_path_ms": round(ms1, 3)}


def bench_window(torch, args, img, tuned):
    """Algorithm 1's own candidate rule (windows around each barycenter) on the
    headline workload, one whole job per step as for the headline."""
    from paper_1903_07149_amd import counts, synth
    from paper_1903_07149_amd._lib import ASSIGN_WINDOW
    from paper_1903_07149_amd.scalp import Scalp

    wl = synth.HD
    H, W = img.contour.shape
    lab = torch.from_numpy(img.lab).cuda()
    con = torch.from_numpy(img.contour).cuda()
    s = Scalp(W, H, wl.k, iterations=wl.iterations, assign_mode=ASSIGN_WINDOW, **tuned)
    out = s.new_state()
    for _ in range(args.warmup):
        s.run(lab, con, out=out)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps // 2)
    t0.record()
    for _ in range(reps):
        s.run(lab, con, out=out)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    g3 = Scalp(W, H, wl.k, iterations=wl.iterations, **tuned).run(lab, con)
    agree = float((out[2] == g3.labels).float().mean().item())
    # algorithmic work of one window pass at the initial grid
    c0, e0, _ = s.init_grid(lab, con)
    R = int(np.floor(np.sqrt(W * H / wl.k) + 0.5))
    flops = counts.window_work(W, H, R, c0.cpu().numpy(), e0.cpu().numpy())["flops"]
    roof = alu_roofline(flops, ms * 1e-3 / wl.iterations,
                        "run / iterations (pack, init, then per iteration the window "
                        "assignment, the sums, finalize and projection); work at the initial grid")
    return {"workload": f"{wl.name}, window of Algorithm 1", "roofline": roof, "mpx_iter_s":
            round(W * H * wl.iterations / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 3),
            "label_agreement_with_3x3_form": round(agree, 4)}


def _time(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def bench_multiscale(torch, args, tuned):
    """Twelve decompositions (6 to 600 superpixels) of the 481x321 image as one
    ragged batch, then their boundary-frequency map: the input of the
    precision-recall evaluation of Sec. III-A.2."""
    from paper_1903_07149_amd import synth
    from paper_1903_07149_amd.maps import MultiScale, boundary_map

    from paper_1903_07149_amd import autotune
    from paper_1903_07149_amd.maps import scales

    img = synth.workload_image(synth.BSD_SHAPE)
    H, W = img.contour.shape
    ks = scales()
    lab_b, con_b = MultiScale.stack_of(len(ks), torch.from_numpy(img.lab).cuda(),
                                       torch.from_numpy(img.contour).cuda())
    # launch shape of the persistent kernel, tuned on this batch of 12 scales
    if args.batch_launch:
        tuned_ms = batch_launch(args.batch_launch)
    else:
        tuned_ms = autotune.tune_batch([(W, H, k) for k in ks], lab_b, con_b, use_cache=False)
    log(f"multiscale launch shape: {tuned_ms}")
    ms = MultiScale(W, H, ks, **tuned_ms)
    state = ms.batch.new_state()
    n = len(ms.ks)

    def step():
        ms.batch.run(lab_b, con_b, out=state)
        boundary_map(state[2].reshape(n, H, W))

    ms_step = _time(torch, step, max(2, args.steps))
    return {"workload": f"481x321, k in {ms.ks}, 10 iterations, one batch + boundary map",
            "launch": tuned_ms, "ms_per_image": round(ms_step, 3), "images_per_s": round(1e3 / ms_step, 1),
            "mpx_iter_s": round(n * W * H * 10 / (ms_step * 1e-3) / 1e6, 1)}


def bench_contour(torch, args, img):
    """The contour prior computed on the device (normalised gradient
    magnitude), standalone and fused into the packing step, on 1920x1080."""
    from paper_1903_07149_amd import synth
    from paper_1903_07149_amd._lib import CONTOUR_GRADIENT
    from paper_1903_07149_amd.maps import contour_from_lab
    from paper_1903_07149_amd.scalp import Scalp

    H, W = img.contour.shape
    N = W * H
    lab = torch.from_numpy(img.lab).cuda()
    con = torch.from_numpy(img.contour).cuda()
    given = Scalp(W, H, synth.HD.k)
    fused = Scalp(W, H, synth.HD.k, contour_source=CONTOUR_GRADIENT)
    reps = max(5, args.steps)
    t_map = _time(torch, lambda: contour_from_lab(lab), reps)
    t_given = _time(torch, lambda: given.prepare(lab, con), reps)
    t_fused = _time(torch, lambda: fused.prepare(lab, None), reps)
    # algorithmic bytes: the map reads lab twice (max, then values) and writes
    # C; plain packing reads lab and C and writes (l, a, b, w); fused packing
    # reads lab twice and writes (l, a, b, w)
    gbs = lambda b, ms: round(b / (ms * 1e-3) / 1e9, 1)
    return {"workload": "1920x1080",
            "contour_map_ms": round(t_map, 4), "contour_map_GBps": gbs(28 * N, t_map),
            "pack_given_prior_ms": round(t_given, 4), "pack_given_prior_GBps": gbs(32 * N, t_given),
            "pack_computed_prior_ms": round(t_fused, 4),
            "pack_computed_prior_GBps": gbs(40 * N, t_fused),
            "two_step_ms": round(t_map + t_given, 4)}


def quality(torch, tuned):
    """Sec. III-A.2 metrics against the synthetic ground truth for the distance
    settings of Sec. III-B, on the 481x321 workload (k = 250, 10 iterations)."""
    from paper_1903_07149_amd import synth
    from paper_1903_07149_amd.metrics import metrics
    from paper_1903_07149_amd.scalp import Scalp

    img = synth.workload_image(synth.BSD_SHAPE)
    H, W = img.contour.shape
    lab = torch.from_numpy(img.lab).cuda()
    con = torch.from_numpy(img.contour).cuda()
    gt = torch.from_numpy(img.gt).cuda()
    out = {}
    for name, kw in [("slic", dict(lam=1.0, gamma=0.0)), ("path_colour", dict(lam=0.5, gamma=0.0)),
                     ("contour", dict(lam=1.0)), ("scalp", dict())]:
        s = Scalp(W, H, 250, **kw, **tuned)
        r = s.run(lab, con)
        m = metrics(r.labels, gt, num_sp=s.K)
        out[name] = {k: round(v, 4) for k, v in m.items() if k in ("br", "asa", "ue", "co")}
    # the same ablation where boundary recall does not saturate: 300
    # ground-truth regions against 250 superpixels; boundary precision is the
    # recall with the two maps swapped, f their F-measure
    fine = synth.make_image(W, H, 300, 10.0, 1)
    flab, fcon, fgt = (torch.from_numpy(a).cuda() for a in (fine.lab, fine.contour, fine.gt))
    R = int(fine.gt.max()) + 1
    out["fine_gt_300_regions"] = {}
    for name, kw in [("slic", dict(lam=1.0, gamma=0.0)), ("path_colour", dict(lam=0.5, gamma=0.0)),
                     ("contour", dict(lam=1.0)), ("scalp", dict())]:
        s = Scalp(W, H, 250, **kw, **tuned)
        r = s.run(flab, fcon)
        m = metrics(r.labels, fgt, num_sp=s.K, num_regions=R)
        bp = metrics(fgt, r.labels, num_sp=R, num_regions=s.K)["br"]
        f = 2 * bp * m["br"] / (bp + m["br"])
        out["fine_gt_300_regions"][name] = {"br": round(m["br"], 4), "bp": round(bp, 4),
                                            "f": round(f, 4), "asa": round(m["asa"], 4),
                                            "ue": round(m["ue"], 4), "co": round(m["co"], 4)}
    # the metric kernels themselves, on the 1920x1080 workload's SCALP labels
    # against its 400-region ground truth
    from paper_1903_07149_amd.metrics import Metrics
    hd = synth.workload_image(synth.HD)
    Hh, Wh = hd.contour.shape
    s = Scalp(Wh, Hh, synth.HD.k, **tuned)
    r = s.run(torch.from_numpy(hd.lab).cuda(), torch.from_numpy(hd.contour).cuda())
    gth = torch.from_numpy(hd.gt).cuda()
    mk = Metrics(Wh, Hh, s.K, int(hd.gt.max()) + 1)
    ms = _time(torch, lambda: mk.run(r.labels, gth), 20)
    out["metrics_1920x1080"] = {"ms": round(ms, 4),
                                "mpx_s": round(Wh * Hh / (ms * 1e-3) / 1e6, 1),
                                "regions": int(hd.gt.max()) + 1, "num_sp": s.K}
    return out


def bench_soft(torch, args):
    from paper_1903_07149_amd import synth
    from paper_1903_07149_amd.scalp import Scalp
    from paper_1903_07149_amd.soft import SoftScalp

    wls = synth.soft_workloads()
    imgs = [synth.workload_image(w) for w in wls]
    B, H, W, k, iters, T = len(wls), wls[0].height, wls[0].width, wls[0].k, wls[0].iterations, 0.5
    lab = torch.from_numpy(np.stack([i.lab for i in imgs])).cuda()
    con = torch.from_numpy(np.stack([i.contour for i in imgs])).cuda()
    gen = torch.Generator(device="cuda").manual_seed(0)
    gq = torch.randn((B, 9, H, W), device="cuda", generator=gen)
    K = SoftScalp(W, H, k, 1, temperature=T, iterations=1).K
    gth = torch.randn((B, K, 5), device="cuda", generator=gen)

    def fwd_bwd_ms(e):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        c_t, q_t, saved = e.forward(lab, con)
        e.backward(lab, con, c_t, q_t, saved, gq, gth)
        t1.record()
        torch.cuda.synchronize()
        return t0.elapsed_time(t1)

    # workgroup size of the soft path kernels: timed once per candidate
    shapes = []
    for wg in (256, 512, 1024):
        e = SoftScalp(W, H, k, B, temperature=T, iterations=iters, wg_size=wg)
        fwd_bwd_ms(e)
        shapes.append((fwd_bwd_ms(e), wg))
        del e
    soft_wg = min(shapes)[1]
    eng = SoftScalp(W, H, k, B, temperature=T, iterations=iters, wg_size=soft_wg)
    for _ in range(2):
        c_t, q_t, saved = eng.forward(lab, con)
        eng.backward(lab, con, c_t, q_t, saved, gq, gth)
    torch.cuda.synchronize()
    reps = 5
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
    for r in range(reps):
        ev[r][0].record()
        c_t, q_t, saved = eng.forward(lab, con)
        ev[r][1].record()
        eng.backward(lab, con, c_t, q_t, saved, gq, gth)
        ev[r][2].record()
    torch.cuda.synchronize()
    fwd = sum(e[0].elapsed_time(e[1]) for e in ev) / reps
    bwd = sum(e[1].elapsed_time(e[2]) for e in ev) / reps
    # the hard path on the same 16 images: one by one (same k and iterations)
    s = Scalp(W, H, k, iterations=iters)
    outs = [s.new_state() for _ in range(B)]
    for b in range(B):
        s.run(lab[b], con[b], out=outs[b])
    torch.cuda.synchronize()
    h0 = torch.cuda.Event(enable_timing=True)
    h1 = torch.cuda.Event(enable_timing=True)
    h0.record()
    for _ in range(reps):
        for b in range(B):
            s.run(lab[b], con[b], out=outs[b])
    h1.record()
    torch.cuda.synchronize()
    hard = h0.elapsed_time(h1) / reps
    # ... and as one ragged batch (persistent launch, shape tuned on it)
    from paper_1903_07149_amd import autotune
    from paper_1903_07149_amd.scalp import ScalpBatch
    shapes = [(W, H, k)] * B
    lab_b, con_b = lab.reshape(-1, 3), con.reshape(-1)
    if args.batch_launch:
        tuned_b = batch_launch(args.batch_launch)
    else:
        tuned_b = autotune.tune_batch(shapes, lab_b, con_b, use_cache=False)
    hb = ScalpBatch(shapes, iterations=iters, **tuned_b)
    hout = hb.new_state()
    hb.run(lab_b, con_b, out=hout)
    torch.cuda.synchronize()
    h0.record()
    for _ in range(reps):
        hb.run(lab_b, con_b, out=hout)
    h1.record()
    torch.cuda.synchronize()
    hard_b = h0.elapsed_time(h1) / reps
    px_it = B * H * W * iters
    # algorithmic work of one soft assignment pass (every slot's path) at the
    # endpoints of Theta_0
    from paper_1903_07149_amd import counts
    th0 = c_t[0].cpu().numpy()
    e0 = np.clip(np.floor(th0[..., 3:5] + np.float32(0.5)), 0, [W - 1, H - 1]).astype(np.int64)
    g = eng.grid
    flops = sum(counts.pass_work(W, H, g.nx, g.ny, e0[bb])["flops"] for bb in range(B))
    roof = alu_roofline(flops, fwd * 1e-3 / iters,
                        "forward / iterations (soft assignment, softmax and soft update); "
                        "work at Theta_0")
    # the backward's: per iteration, a pair re-walks its path to that
    # iteration's endpoint when its dL/dD is not zero: Q >= 2^-24 at a pixel
    # whose Q is not one-hot in FP32 (where the largest Q is exactly 1, the
    # softmax backward G_j - sum_i Q_i G_i rounds to 0); the last timed
    # forward's Q and Theta
    bflops = 0
    bsamples = 0
    for t in range(iters):
        qt = q_t[t]
        walked = ((qt >= 2.0 ** -24) & (qt.amax(dim=1, keepdim=True) < 1.0)).cpu().numpy()
        tht = c_t[t].cpu().numpy()
        et = np.clip(np.floor(tht[..., 3:5] + np.float32(0.5)), 0, [W - 1, H - 1]).astype(np.int64)
        for bb in range(B):
            w = counts.soft_backward_work(W, H, g.nx, g.ny, et[bb], walked[bb])
            bflops += w["flops"]
            bsamples += w["samples"]
    roof_b = alu_roofline(bflops / iters, bwd * 1e-3 / iters,
                          "backward / iterations (softmax and soft-update backward, and the "
                          "path re-walk of every pair whose dL/dD is not zero); work at every "
                          "iteration's Q")
    roof_b["walked_samples_per_iteration"] = int(bsamples // iters)
    return {"workload": f"{B} x {W}x{H} Voronoi images, k={k}, T={T}, {iters} iterations",
            "roofline_forward": roof,
            "roofline_backward": roof_b,
            "wg_size": soft_wg,
            "fwd_bwd_mpx_iter_s": round(px_it / ((fwd + bwd) * 1e-3) / 1e6, 1),
            "fwd_ms": round(fwd, 3), "bwd_ms": round(bwd, 3),
            "fwd_mpx_iter_s": round(px_it / (fwd * 1e-3) / 1e6, 1),
            "hard_same_images_mpx_iter_s": round(px_it / (hard * 1e-3) / 1e6, 1),
            "hard_same_images_ms": round(hard, 3),
            "hard_same_images_batched_mpx_iter_s": round(px_it / (hard_b * 1e-3) / 1e6, 1),
            "hard_same_images_batched_ms": round(hard_b, 3),
            "hard_same_images_batched_launch": tuned_b}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the batched and "
              "single-image paths shard by image across GPUs without communication, so "
              "per-GPU throughput is the figure", file=sys.stderr)
        sys.exit(2)
    if args.extensions is not None:
        unknown = set(args.extensions.split(",")) - set(EXTENSIONS)
        if unknown:
            print(f"unknown extensions: {sorted(unknown)}", file=sys.stderr)
            sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU (torch.cuda.is_available() is False)", file=sys.stderr)
        sys.exit(1)
    log("hard SCALP, 1920x1080, k=2000, 10 iterations")
    img, tuned, hard = bench_hard(torch, args)
    out = {
        "metric": METRIC, "value": round(hard["value"], 1), "unit": "Mpixel-iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(hard["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": hard["config"], "roofline": hard["roofline"],
        "eager_ms_per_step": round(hard["eager_ms_per_step"], 4),
        "eager_value": round(hard["eager_value"], 1),
        "without_pruning": hard["without_pruning"],
    }
    if not args.no_extensions:
        runs = [("batched", lambda: bench_batched(torch, args, tuned)),
                ("soft", lambda: bench_soft(torch, args)),
                ("window_form", lambda: bench_window(torch, args, img, tuned)),
                ("multiscale", lambda: bench_multiscale(torch, args, tuned)),
                ("contour_prior", lambda: bench_contour(torch, args, img)),
                ("quality", lambda: quality(torch, tuned))]
        want = None if args.extensions is None else set(args.extensions.split(","))
        names = {"multiscale": "multiscale_481x321", "quality": "quality_481x321"}
        out["extensions"] = {}
        for name, fn in runs:
            if want is None or name in want:
                log(name)
                out["extensions"][names.get(name, name)] = fn()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(img, 2000, 10)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
