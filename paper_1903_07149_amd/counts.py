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


def window_work(width: int, height: int, radius: int, centres: np.ndarray,
                endpoints: np.ndarray) -> dict:
    """samples, candidates, flops of one pass of the window form: every pixel of
    every cluster's (2R+1)^2 window (around its barycenter rounded to a pixel,
    clamped into the image, clipped by the borders) walks its path to the
    cluster's endpoint."""
    W, H, R = int(width), int(height), int(radius)
    c = np.asarray(centres, np.float32).reshape(-1, 5)
    ep = np.asarray(endpoints, np.int64).reshape(-1, 2)
    wx = np.clip(np.floor(c[:, 3] + np.float32(0.5)).astype(np.int64), 0, W - 1)
    wy = np.clip(np.floor(c[:, 4] + np.float32(0.5)).astype(np.int64), 0, H - 1)
    samples = 0
    cands = 0
    for k in range(ep.shape[0]):
        xs = np.arange(max(0, wx[k] - R), min(W, wx[k] + R + 1))
        ys = np.arange(max(0, wy[k] - R), min(H, wy[k] + R + 1))
        n = np.maximum(np.abs(ep[k, 0] - xs)[None, :], np.abs(ep[k, 1] - ys)[:, None])
        samples += int((n + 1).sum())
        cands += n.size
    return {"samples": samples, "candidates": cands,
            "flops": FLOPS_PER_SAMPLE * samples + FLOPS_PER_CANDIDATE * cands,
            "lds_bytes": BYTES_PER_SAMPLE * samples}


# The soft backward, per iteration: every (pixel, slot) pair whose softmax
# weight is at least 2^-24 re-walks its path, and every sample q of it takes
# dL/df_q += cf (f_q - f_k) (3 sub, 3 mul, 3 add), dL/dw_q += cw (1 add) and
# the candidate's centre gradient -cf (f_q - f_k) (3 add); per pair the two
# weights cf, cw and the spatial part of the centre gradient; per pixel the
# softmax and soft-update backward over its 9 slots (dL/dQ from the two
# candidate terms, its dot with Q, dL/dD, dL/df through the update).
SOFT_BWD_FLOPS_PER_SAMPLE = 13
SOFT_BWD_FLOPS_PER_PAIR = 14
SOFT_BWD_FLOPS_PER_PIXEL = 9 * 19


def soft_backward_work(width: int, height: int, nx: int, ny: int, endpoints: np.ndarray,
                       walked: np.ndarray) -> dict:
    """samples, pairs, flops of one soft backward iteration of one image.
    endpoints: [K'][2] (x, y) of the iteration's candidate endpoints;
    walked: bool [9][H][W] (slot-major, slot j = 3 (di + 1) + (dj + 1) of the
    pixel's cell offset), True where the pair's path is re-walked."""
    W, H = int(width), int(height)
    yy, xx = np.mgrid[0:H, 0:W]
    ci = (yy.astype(np.int64) * ny) // H
    cj = (xx.astype(np.int64) * nx) // W
    ep = np.asarray(endpoints, np.int64).reshape(-1, 2)
    wk = np.asarray(walked, bool).reshape(9, H, W)
    samples = 0
    pairs = 0
    for j in range(9):
        ii, jj = ci + j // 3 - 1, cj + j % 3 - 1
        ok = (ii >= 0) & (ii < ny) & (jj >= 0) & (jj < nx) & wk[j]
        k = np.where(ok, ii * nx + jj, 0)
        n = np.maximum(np.abs(ep[k, 0] - xx), np.abs(ep[k, 1] - yy))
        samples += int(((n + 1) * ok).sum())
        pairs += int(ok.sum())
    return {"samples": samples, "pairs": pairs,
            "flops": SOFT_BWD_FLOPS_PER_SAMPLE * samples + SOFT_BWD_FLOPS_PER_PAIR * pairs +
                     SOFT_BWD_FLOPS_PER_PIXEL * W * H}
