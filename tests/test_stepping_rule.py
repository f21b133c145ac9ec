"""The assignment kernels step along a linear path by counting the carries of
a 32-bit accumulator (start 2^31, increment F = ceil(2^32 |d_minor| / n), or
2^32 - 1 for a diagonal).  This checks, on the CPU, that the carry count after
i steps equals the path's minor-axis offset floor((2 i |d_minor| + n) / (2 n))
of Sec. II-B for every step: exhaustively for short paths, on random pairs up
to the bound n < 46340 the argument gives."""
import math

import numpy as np
import pytest


def _increment(am: int, n: int) -> int:
    if am == n:
        return 0xFFFFFFFF
    # the same double-precision expression the kernels evaluate
    return int(math.ceil(float(am) * 4294967296.0 / float(n)))


def _check(n: int, am: int) -> None:
    i = np.arange(1, n, dtype=np.uint64)
    F = np.uint64(_increment(am, n))
    carries = (np.uint64(1 << 31) + i * F) >> np.uint64(32)
    exact = (2 * i.astype(np.int64) * am + n) // (2 * n)
    assert (carries.astype(np.int64) == exact).all(), (n, am)


def test_exhaustive_short_paths():
    for n in range(2, 257):
        for am in range(0, n + 1):
            _check(n, am)


@pytest.mark.parametrize("seed", range(4))
def test_random_long_paths(seed):
    rng = np.random.default_rng(seed)
    for n in rng.integers(257, 46340, 40):
        n = int(n)
        for am in (0, 1, n // 3, n // 2, n - 1, n, int(rng.integers(0, n + 1))):
            _check(n, am)


def test_ties_round_toward_the_endpoint():
    # n = 4, |d_minor| = 2: the segment passes exactly between two pixels at
    # i = 1 and i = 3 (i s = 1/2, 3/2); offsets floor((4 i + 4) / 8) = 1, 1, 2
    # take the pixel nearer the endpoint
    F = _increment(2, 4)
    assert [((1 << 31) + i * F) >> 32 for i in (1, 2, 3)] == [1, 1, 2]
