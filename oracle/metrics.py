"""Plain numpy definitions of the superpixel quality metrics of Sec. III-A.2
(test infrastructure only, like the rest of the oracle package).

Readings (the paper gives the formulas, not these details):
  * boundary pixels B(S): pixels with at least one 4-connected neighbour
    inside the image carrying a different label;
  * BR, Eq. (5): fraction of ground-truth boundary pixels p with a
    superpixel boundary pixel q at Euclidean distance ||p - q|| < epsilon
    (epsilon = 2: the 3x3 neighbourhood of p); 1 when the ground truth has no
    boundary pixel;
  * ASA, Eq. (6): sum over superpixels of the largest overlap with one
    ground-truth region, over the number of pixels;
  * UE, Eq. (7): sum over regions G_i and superpixels S_k meeting G_i of
    |S_k - G_i| = |S_k| - |S_k n G_i|, over the number of pixels;
  * CO, Eq. (8): (1/|I|) sum_k 4 pi |S_k|^2 / |P(S_k)|^2 with |P(S_k)| the
    number of pixel edges between S_k and another label or the image border
    (4-connectivity); empty superpixels are skipped.
"""
from __future__ import annotations

import math

import numpy as np


def boundary(labels: np.ndarray) -> np.ndarray:
    L = np.asarray(labels)
    b = np.zeros(L.shape, bool)
    d = L[:, 1:] != L[:, :-1]
    b[:, 1:] |= d
    b[:, :-1] |= d
    d = L[1:, :] != L[:-1, :]
    b[1:, :] |= d
    b[:-1, :] |= d
    return b


def boundary_recall(sp: np.ndarray, gt: np.ndarray, eps: float = 2.0) -> float:
    bs = boundary(sp)
    bg = boundary(gt)
    n = int(bg.sum())
    if n == 0:
        return 1.0
    H, W = bs.shape
    r = int(math.ceil(eps)) - 1
    near = np.zeros_like(bs)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            if dx * dx + dy * dy >= eps * eps:
                continue
            src = bs[max(0, dy):H + min(0, dy), max(0, dx):W + min(0, dx)]
            near[max(0, -dy):H + min(0, -dy), max(0, -dx):W + min(0, -dx)] |= src
    return float((near & bg).sum()) / n


def overlap_table(sp: np.ndarray, gt: np.ndarray):
    s = np.asarray(sp).ravel().astype(np.int64)
    g = np.asarray(gt).ravel().astype(np.int64)
    K = int(s.max()) + 1
    R = int(g.max()) + 1
    t = np.bincount(s * R + g, minlength=K * R).reshape(K, R)
    return t


def asa(sp: np.ndarray, gt: np.ndarray) -> float:
    t = overlap_table(sp, gt)
    return float(t.max(axis=1).sum()) / np.asarray(sp).size


def undersegmentation_error(sp: np.ndarray, gt: np.ndarray) -> float:
    t = overlap_table(sp, gt)
    size = t.sum(axis=1, keepdims=True)
    return float(((size - t) * (t > 0)).sum()) / np.asarray(sp).size


def perimeters(sp: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    L = np.asarray(sp).astype(np.int64)
    K = int(L.max()) + 1
    area = np.bincount(L.ravel(), minlength=K)
    H, W = L.shape
    edges = np.zeros(K, np.int64)
    # image border edges
    edges += np.bincount(L[0, :], minlength=K) + np.bincount(L[-1, :], minlength=K)
    edges += np.bincount(L[:, 0], minlength=K) + np.bincount(L[:, -1], minlength=K)
    # inner edges, counted for both sides
    d = L[:, 1:] != L[:, :-1]
    edges += np.bincount(L[:, 1:][d], minlength=K) + np.bincount(L[:, :-1][d], minlength=K)
    d = L[1:, :] != L[:-1, :]
    edges += np.bincount(L[1:, :][d], minlength=K) + np.bincount(L[:-1, :][d], minlength=K)
    return area, edges


def compactness(sp: np.ndarray) -> float:
    area, per = perimeters(sp)
    nz = area > 0
    a = area[nz].astype(np.float64)
    p = per[nz].astype(np.float64)
    return float((4.0 * math.pi * a * a / (p * p)).sum()) / np.asarray(sp).size


def all_metrics(sp: np.ndarray, gt: np.ndarray, eps: float = 2.0) -> dict:
    return {"br": boundary_recall(sp, gt, eps), "asa": asa(sp, gt),
            "ue": undersegmentation_error(sp, gt), "co": compactness(sp)}
