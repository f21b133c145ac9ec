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
