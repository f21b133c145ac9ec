"""Plain numpy definitions of two per-pixel maps (test infrastructure only,
like the rest of the oracle package; the product path never imports it).

boundary_frequency
    The multi-scale boundary map behind the precision-recall evaluation of
    Sec. III-A.2: several decompositions of one image (the paper uses 12
    scales from 6 to 600 superpixels) are turned into one soft boundary map,
    the fraction of decompositions in which a pixel lies on a superpixel
    boundary.  Reading: a boundary pixel is one with a 4-neighbour inside the
    image carrying another label; the fraction is c / n rounded to FP32.

contour_prior
    A soft contour map C in [0, 1] (Sec. II-D) computed from the image
    itself, standing in for the learned detectors of Sec. II-E.  Reading: the
    central-difference gradient g = (f(x+1) - f(x-1)) / 2 in x and in y of
    every Lab channel, borders replicated, magnitude sqrt(sum over channels
    of gx^2 + gy^2), divided by its largest value over the image; FP64, one
    rounding to FP32 at the end; a constant image gives zeros.
"""
from __future__ import annotations

import numpy as np


def boundary_frequency(labels: np.ndarray) -> np.ndarray:
    """labels: int [n][H][W] -> float32 [H][W]."""
    L = np.asarray(labels)
    n, H, W = L.shape
    count = np.zeros((H, W), np.int64)
    for s in range(n):
        M = L[s]
        b = np.zeros((H, W), bool)
        if W > 1:
            d = M[:, 1:] != M[:, :-1]     # horizontal neighbours differ
            b[:, 1:] |= d
            b[:, :-1] |= d
        if H > 1:
            d = M[1:, :] != M[:-1, :]     # vertical neighbours differ
            b[1:, :] |= d
            b[:-1, :] |= d
        count += b
    return (count.astype(np.float32) / np.float32(n)).astype(np.float32)


def gradient_magnitude(lab: np.ndarray) -> np.ndarray:
    """lab: float [H][W][3] -> float64 [H][W], unnormalised."""
    f = np.asarray(lab, np.float64)
    H, W, _ = f.shape
    xs = np.arange(W)
    ys = np.arange(H)
    right = f[:, np.minimum(xs + 1, W - 1), :]
    left = f[:, np.maximum(xs - 1, 0), :]
    down = f[np.minimum(ys + 1, H - 1), :, :]
    up = f[np.maximum(ys - 1, 0), :, :]
    gx = 0.5 * (right - left)
    gy = 0.5 * (down - up)
    per_channel = gx * gx + gy * gy
    total = per_channel[..., 0]
    for c in (1, 2):                      # channels summed in order
        total = total + per_channel[..., c]
    return np.sqrt(total)


def contour_prior(lab: np.ndarray) -> np.ndarray:
    """lab: float [H][W][3] -> float32 [H][W] in [0, 1]."""
    g = gradient_magnitude(lab)
    m = float(g.max()) if g.size else 0.0
    if m > 0.0:
        return (g / m).astype(np.float32)
    return np.zeros(g.shape, np.float32)
