"""Pins for the numpy metric definitions (Eqs. (5)-(8)) by closed forms and a
brute-force boundary recall."""
import math

import numpy as np
import pytest

from oracle import metrics as M


def test_identical_partition():
    rng = np.random.default_rng(0)
    g = rng.integers(0, 7, (30, 40))
    assert M.boundary_recall(g, g) == 1.0
    assert M.asa(g, g) == 1.0
    assert M.undersegmentation_error(g, g) == 0.0


def test_single_superpixel():
    g = np.zeros((20, 30), np.int64)
    g[:, 10:] = 1
    g[12:, 20:] = 2
    s = np.zeros_like(g)
    sizes = np.bincount(g.ravel())
    assert M.asa(s, g) == sizes.max() / g.size
    assert math.isclose(M.undersegmentation_error(s, g), (3 * g.size - g.size) / g.size)
    assert M.boundary_recall(s, g) == 0.0


def test_compactness_closed_forms():
    a = 8
    sq = (np.arange(32)[:, None] // a) * 4 + (np.arange(32)[None, :] // a)   # 4x4 squares
    assert math.isclose(M.compactness(sq), math.pi / 4)
    row = np.zeros((1, 50), np.int64)
    assert math.isclose(M.compactness(row), 4 * math.pi * 50 ** 2 / (2 * 50 + 2) ** 2 / 50)
    area, per = M.perimeters(sq)
    assert (area == 64).all() and (per == 32).all()


@pytest.mark.parametrize("shift,expected", [(0, 1.0), (1, 1.0), (2, 0.5), (3, 0.0)])
def test_boundary_recall_tolerance(shift, expected):
    g = np.zeros((10, 40), np.int64)
    g[:, 20:] = 1
    s = np.zeros_like(g)
    s[:, 20 + shift:] = 1
    assert M.boundary_recall(s, g, eps=2.0) == expected


@pytest.mark.parametrize("eps", [1.0, 2.0, 3.5, 5.0])
def test_boundary_recall_brute_force_blocky(eps):
    """Sparse boundaries (blocky maps) so that the tolerance decides: for
    eps = 5 the offsets (3, 4) lie exactly at distance eps and do not count."""
    rng = np.random.default_rng(int(eps * 10))
    H, W = 30, 33
    for _ in range(3):
        g = np.kron(rng.integers(0, 4, (H // 6 + 1, W // 6 + 1)), np.ones((6, 6), np.int64))[:H, :W]
        s = np.kron(rng.integers(0, 5, (H // 5 + 1, W // 5 + 1)), np.ones((5, 5), np.int64))[:H, :W]
        s = np.roll(s, (2, 3), axis=(0, 1))
        bg, bs = M.boundary(g), M.boundary(s)
        qs = np.argwhere(bs)
        hits = 0
        for y, x in np.argwhere(bg):
            d2 = (qs[:, 0] - y) ** 2 + (qs[:, 1] - x) ** 2
            hits += bool((d2 < eps * eps).any())
        got = M.boundary_recall(s, g, eps)
        assert math.isclose(got, hits / bg.sum())
        assert 0.0 < got < 1.0 or eps >= 3.5


def test_boundary_recall_at_the_tolerance():
    """Two one-pixel islands, ground truth at (10, 10) and superpixel at
    (14, 14): each boundary is the island and its 4 neighbours.  With eps = 5
    the ground-truth pixels (11, 10) and (10, 11) are at distance sqrt(20)
    from (13, 14) / (14, 13); (10, 10) is at exactly 5 (offsets (3, 4) and
    (4, 3)) and does not count; (9, 10) and (10, 9) are farther.  BR = 2/5."""
    g = np.zeros((30, 30), np.int64)
    g[10, 10] = 1
    s = np.zeros_like(g)
    s[14, 14] = 1
    assert M.boundary_recall(s, g, eps=5.0) == 2 / 5
    assert M.boundary_recall(s, g, eps=5.0 + 1e-9) == 3 / 5


def test_boundary_recall_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(5):
        g = rng.integers(0, 3, (12, 15))
        s = rng.integers(0, 4, (12, 15))
        bg, bs = M.boundary(g), M.boundary(s)
        for y in range(12):
            for x in range(15):
                nb = [s[y + dy, x + dx] != s[y, x] for dy, dx in ((0, 1), (1, 0), (0, -1), (-1, 0))
                      if 0 <= y + dy < 12 and 0 <= x + dx < 15]
                assert bs[y, x] == any(nb)
        hits = 0
        for y, x in zip(*np.nonzero(bg)):
            qs = list(zip(*np.nonzero(bs)))
            hits += any((qy - y) ** 2 + (qx - x) ** 2 < 4 for qy, qx in qs)
        assert math.isclose(M.boundary_recall(s, g), hits / bg.sum())
