"""Pins for the oracle's linear path (Sec. II-B: Bresenham pixels from p to
the superpixel barycenter).

The oracle uses a closed form indexed by the step i.  It is checked against
two independent definitions of the same digital line:
  * the textbook incremental Bresenham error-term algorithm, written here for
    every octant, stepping the minor axis when the decision variable is >= 0;
  * the exact nearest-integer rule with rational arithmetic: on major-axis
    step i the minor coordinate is the integer nearest to the real segment,
    ties taken toward the endpoint.
"""
from fractions import Fraction

import numpy as np
import pytest


def bresenham_incremental(x0, y0, x1, y1):
    dx, dy = x1 - x0, y1 - y0
    sx = 1 if dx > 0 else -1
    sy = 1 if dy > 0 else -1
    adx, ady = abs(dx), abs(dy)
    x, y = x0, y0
    pts = [(x, y)]
    if adx >= ady:
        e = 2 * ady - adx
        for _ in range(adx):
            if e >= 0 and ady > 0:
                y += sy
                e -= 2 * adx
            e += 2 * ady
            x += sx
            pts.append((x, y))
    else:
        e = 2 * adx - ady
        for _ in range(ady):
            if e >= 0 and adx > 0:
                x += sx
                e -= 2 * ady
            e += 2 * adx
            y += sy
            pts.append((x, y))
    return pts


def nearest_rational(x0, y0, x1, y1):
    dx, dy = x1 - x0, y1 - y0
    n = max(abs(dx), abs(dy))
    if n == 0:
        return [(x0, y0)]

    def rnd(v: Fraction, toward_positive: bool) -> int:
        fl = v.numerator // v.denominator
        frac = v - fl
        if frac > Fraction(1, 2) or (frac == Fraction(1, 2) and toward_positive):
            return fl + 1
        return fl

    pts = []
    for i in range(n + 1):
        t = Fraction(i, n)
        px = rnd(x0 + t * dx, dx > 0)
        py = rnd(y0 + t * dy, dy > 0)
        pts.append((px, py))
    return pts


def test_small_known_path(orc):
    # (0,0) -> (5,2): minor coordinate 2i/5 = 0.4, 0.8, 1.2, 1.6, 2.0 rounds to 0,1,1,2,2
    assert orc.path(0, 0, 5, 2).tolist() == [[0, 0], [1, 0], [2, 1], [3, 1], [4, 2], [5, 2]]
    # exact half: (0,0) -> (2,1) has minor 0.5 at i=1, rounded toward the endpoint
    assert orc.path(0, 0, 2, 1).tolist() == [[0, 0], [1, 1], [2, 1]]
    assert orc.path(2, 1, 0, 0).tolist() == [[2, 1], [1, 0], [0, 0]]
    assert orc.path(3, 3, 3, 3).tolist() == [[3, 3]]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_three_definitions_agree(orc, seed):
    rng = np.random.default_rng(seed)
    for _ in range(1500):
        x0, y0, x1, y1 = (int(v) for v in rng.integers(-40, 41, 4))
        got = [tuple(p) for p in orc.path(x0, y0, x1, y1).tolist()]
        assert got == bresenham_incremental(x0, y0, x1, y1)
        assert got == nearest_rational(x0, y0, x1, y1)


def test_path_properties(orc):
    rng = np.random.default_rng(7)
    for _ in range(2000):
        x0, y0, x1, y1 = (int(v) for v in rng.integers(0, 90, 4))
        p = orc.path(x0, y0, x1, y1)
        n = max(abs(x1 - x0), abs(y1 - y0))
        assert len(p) == n + 1
        assert tuple(p[0]) == (x0, y0) and tuple(p[-1]) == (x1, y1)
        steps = np.abs(np.diff(p, axis=0))
        assert (steps.max(axis=1) == 1).all()          # 8-connected, one pixel per step
        major = 0 if abs(x1 - x0) >= abs(y1 - y0) else 1
        if n:
            assert (steps[:, major] == 1).all()          # one major-axis step per sample
        # inside the bounding box of its ends
        assert p[:, 0].min() >= min(x0, x1) and p[:, 0].max() <= max(x0, x1)
        assert p[:, 1].min() >= min(y0, y1) and p[:, 1].max() <= max(y0, y1)
        # transposing the plane transposes the path
        pt = orc.path(y0, x0, y1, x1)
        assert (pt[:, ::-1] == p).all()
