"""Autotuner for the assignment kernel's launch shape.

Knobs that change speed but never results (every configuration is checked
bit-exact against the oracle by the GPU tests): the workgroup size (lanes
of one work item, one pixel each, sharing its LDS tables), the LDS budget
in 16-byte units (the size of the two per-candidate tables, which bounds
which candidates walk over LDS rather than global memory, and how many
workgroups fit on a CU), the table mode (per-candidate tables over the work
item's rectangle, or voted down to the walking waves' box) and, for a ragged
batch, the number of persistent workgroups per CU.

tune() times one fused assignment pass (`scalp_assign_accumulate`) per
configuration with HIP events on the workload's own image and superpixel
state; tune_batch() times whole batched runs (`scalp_run_batched`: packing,
grid initialisation and two persistent iterations) on the batch itself.
Winners are cached in a JSON file keyed by device architecture and workload
shape (for a batch: the histogram of its images' sizes and cell sides).
"""
from __future__ import annotations

import hashlib
import json
import math
import os

import torch

from .scalp import Scalp, ScalpBatch

CANDIDATES = ([dict(wg_size=w, lds_pixels=p) for w in (256, 512, 1024)
               for p in (1, 2400, 3200, 3840, 4800)] +
              [dict(wg_size=w, lds_pixels=p, table_mode=1) for w in (256, 512, 1024)
               for p in (2400, 4800, 9728)])
BATCH_CANDIDATES = ([dict(wg_size=w, lds_pixels=p, persistent_blocks=b)
                     for w in (256, 512, 1024) for p in (2400, 3840, 4800, 9728)
                     for b in (0, 1, 2)] +
                    [dict(wg_size=w, lds_pixels=p, persistent_blocks=b, table_mode=1)
                     for w in (256, 512, 1024) for p in (2400, 4800, 9728) for b in (0, 1)])
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def _key(width: int, height: int, k: int) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return f"{arch}/{width}x{height}/k{k}"


def time_config(s: Scalp, lab, contour, cfg: dict, reps: int = 5, warm_iters: int = 3) -> float:
    """Average milliseconds of one fused assignment pass with `cfg`, from the
    superpixel state after `warm_iters` iterations."""
    c, e, l, n = s.new_state()
    s.init_grid(lab, contour, out=(c, e, l))
    for _ in range(warm_iters):
        s.assign_accumulate(c, e, l)
        s.finalize(l, c, e, n)
    s.assign_accumulate(c, e, l, **cfg)          # warm-up launch of this shape
    s.finalize(l, c.clone(), e.clone(), n)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        s.assign_accumulate(c, e, l, **cfg)
        b.record()
        s.finalize(l, c.clone(), e.clone(), n)   # clears the sums; state stays fixed
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / reps


def tune(width: int, height: int, k: int, lab, contour, candidates=None, use_cache=True,
         verbose=False) -> dict:
    key = _key(width, height, k)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        with open(CACHE) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["best"]
    s = Scalp(width, height, k)
    results = []
    for cfg in candidates or CANDIDATES:
        ms = time_config(s, lab, contour, cfg)
        results.append((ms, cfg))
        if verbose:
            print(f"[autotune] {key} {cfg}: {ms:.4f} ms")
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    cache[key] = {"best": best, "ms": results[0][0],
                  "all": [{"cfg": c, "ms": m} for m, c in results]}
    if use_cache:
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    return best


def batch_key(shapes) -> str:
    """Cache key of a ragged batch: architecture, image count, and a digest of
    the histogram of (pixel count in half-octaves, cell side r in pixels)."""
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    hist = {}
    for (w, h, k) in shapes:
        n = w * h
        b = (round(2 * math.log2(n)), round(math.sqrt(n / k)))
        hist[b] = hist.get(b, 0) + 1
    text = ";".join(f"{a},{r}:{c}" for (a, r), c in sorted(hist.items()))
    return f"{arch}/batch{len(shapes)}/{hashlib.sha1(text.encode()).hexdigest()[:12]}"


def time_batch_config(shapes, lab, contour, cfg: dict, reps: int = 2, iterations: int = 2) -> float:
    """Average milliseconds of one batched run (pack, init, `iterations`
    persistent iterations) with `cfg`."""
    b = ScalpBatch(shapes, iterations=iterations, **cfg)
    out = b.new_state()
    b.run(lab, contour, out=out)                  # warm-up of this shape
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, e in ev:
        a.record()
        b.run(lab, contour, out=out)
        e.record()
    torch.cuda.synchronize()
    return sum(a.elapsed_time(e) for a, e in ev) / reps


def tune_batch(shapes, lab, contour, candidates=None, use_cache=True, verbose=False) -> dict:
    """Launch shape of scalp_run_batched for this batch (lab [N][3], contour [N]
    concatenated in the order of `shapes`)."""
    key = batch_key(shapes)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        with open(CACHE) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["best"]
    results = []
    for cfg in candidates or BATCH_CANDIDATES:
        ms = time_batch_config(shapes, lab, contour, cfg)
        results.append((ms, cfg))
        if verbose:
            print(f"[autotune] {key} {cfg}: {ms:.4f} ms")
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    cache[key] = {"best": best, "ms": results[0][0],
                  "all": [{"cfg": c, "ms": m} for m, c in results]}
    if use_cache:
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    return best
