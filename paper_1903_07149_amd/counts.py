"""Algorithmic work of one assignment pass (for throughput and roofline
figures): host-side integer geometry only.

For every pixel p and each of its 3x3 grid-neighbour candidates k the
linear path of Sec. II-B from p to k's endpoint has n + 1 samples, with
n = max(|dx|, |dy|).  Per sample the distance of Eqs. (1)-(2) performs
10 FP32 operations (3 sub, 3 mul, 2 add for d_c; 1 add each for the colour
and contour sums) and reads one 16-byte (l, a, b, w) texel; per (pixel,
candidate) the normalisations and Eq. (3) add 16 more (2 divisions, the
spatial term and the comparison).
"""
from __future__ import annotations

import numpy as np

FLOPS_PER_SAMPLE = 10
FLOPS_PER_CANDIDATE = 16
BYTES_PER_SAMPLE = 16


def pass_work(width: int, height: int, nx: int, ny: int, endpoints: np.ndarray) -> dict:
    """samples, candidates, flops of one pass for the given endpoints (K'x2)."""
    W, H = int(width), int(height)
    yy, xx = np.mgrid[0:H, 0:W]
    ci = (yy.astype(np.int64) * ny) // H
    cj = (xx.astype(np.int64) * nx) // W
    ep = np.asarray(endpoints, np.int64).reshape(-1, 2)
    samples = 0
    cands = 0
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            ii, jj = ci + di, cj + dj
            ok = (ii >= 0) & (ii < ny) & (jj >= 0) & (jj < nx)
            k = np.where(ok, ii * nx + jj, 0)
            n = np.maximum(np.abs(ep[k, 0] - xx), np.abs(ep[k, 1] - yy))
            samples += int(((n + 1) * ok).sum())
            cands += int(ok.sum())
    return {"samples": samples, "candidates": cands,
            "flops": FLOPS_PER_SAMPLE * samples + FLOPS_PER_CANDIDATE * cands,
            "lds_bytes": BYTES_PER_SAMPLE * samples}
