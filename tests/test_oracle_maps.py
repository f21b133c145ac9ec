"""Pins of the oracle's per-pixel maps (boundary frequency, contour prior)
against brute force and closed forms."""
import numpy as np
import pytest

from oracle import maps as O


def _brute_boundary(M):
    H, W = M.shape
    out = np.zeros((H, W), bool)
    for y in range(H):
        for x in range(W):
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                qx, qy = x + dx, y + dy
                if 0 <= qx < W and 0 <= qy < H and M[qy, qx] != M[y, x]:
                    out[y, x] = True
    return out


@pytest.mark.parametrize("H,W,n,seed", [(7, 9, 3, 1), (1, 12, 2, 2), (10, 1, 4, 3), (1, 1, 1, 4),
                                        (16, 16, 12, 5)])
def test_boundary_frequency_brute_force(H, W, n, seed):
    rng = np.random.default_rng(seed)
    L = rng.integers(0, 3, (n, H, W)).astype(np.int32)
    got = O.boundary_frequency(L)
    cnt = sum(_brute_boundary(L[s]).astype(np.int64) for s in range(n))
    assert got.dtype == np.float32
    assert (got == (np.asarray(cnt, np.float32) / np.float32(n))).all()


def test_boundary_frequency_special_cases():
    H, W = 6, 8
    const = np.zeros((H, W), np.int32)
    checker = (np.add.outer(np.arange(H), np.arange(W)) % 2).astype(np.int32)
    halves = np.zeros((H, W), np.int32)
    halves[:, W // 2:] = 1
    assert (O.boundary_frequency(const[None]) == 0).all()
    assert (O.boundary_frequency(checker[None]) == 1).all()
    # a vertical split: only the two columns next to it are boundary
    f = O.boundary_frequency(np.stack([halves, const]))
    expect = np.zeros((H, W), np.float32)
    expect[:, W // 2 - 1:W // 2 + 1] = 0.5
    assert (f == expect).all()
    # relabelling a map does not move its boundaries
    assert (O.boundary_frequency((halves * 7 + 3)[None]) == O.boundary_frequency(halves[None])).all()


def _lab(H, W, fn_l=None, fn_a=None, fn_b=None):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    lab = np.zeros((H, W, 3), np.float64)
    for c, fn in enumerate((fn_l, fn_a, fn_b)):
        if fn is not None:
            lab[..., c] = fn(x, y)
    return lab.astype(np.float32)


def test_contour_quadratic_ramp():
    """f = x^2: the central difference is 2x inside, 1/2 at x = 0 and
    (2W - 3)/2 at x = W - 1; the largest value is 2(W - 2)."""
    H, W = 5, 11
    g = O.gradient_magnitude(_lab(H, W, fn_l=lambda x, y: x * x))
    x = np.arange(W, dtype=np.float64)
    expect = 2.0 * x
    expect[0] = 0.5
    expect[-1] = (2 * W - 3) / 2.0
    assert np.array_equal(g, np.broadcast_to(expect, (H, W)))
    c = O.contour_prior(_lab(H, W, fn_l=lambda x, y: x * x))
    assert np.array_equal(c, np.broadcast_to((expect / (2.0 * (W - 2))).astype(np.float32), (H, W)))
    assert c.max() == 1.0


def test_contour_step_edge_and_channels():
    """A step of height h in one channel: magnitude h/2 on the two pixels
    beside it, 0 elsewhere; the same step in two channels scales by sqrt 2."""
    H, W, h = 4, 10, 6.0
    one = O.gradient_magnitude(_lab(H, W, fn_a=lambda x, y: h * (x >= 5)))
    assert np.array_equal(one[:, 4:6], np.full((H, 2), h / 2))
    assert (np.delete(one, [4, 5], axis=1) == 0).all()
    two = O.gradient_magnitude(_lab(H, W, fn_a=lambda x, y: h * (x >= 5), fn_b=lambda x, y: h * (x >= 5)))
    assert np.allclose(two, np.sqrt(2.0) * one, rtol=0, atol=1e-12)
    assert np.array_equal(O.contour_prior(_lab(H, W, fn_a=lambda x, y: h * (x >= 5))),
                          (one / (h / 2)).astype(np.float32))


def test_contour_plane_and_symmetry():
    """f = 3x + 4y: |g| = 5 inside; x and y swap under transposition."""
    H, W = 7, 9
    g = O.gradient_magnitude(_lab(H, W, fn_b=lambda x, y: 3 * x + 4 * y))
    assert np.allclose(g[1:-1, 1:-1], 5.0, rtol=0, atol=1e-12)
    # border: one-sided half differences, e.g. the left column has gx = 1.5
    assert np.allclose(g[1:-1, 0], np.hypot(1.5, 4.0), rtol=0, atol=1e-12)
    rng = np.random.default_rng(7)
    lab = rng.normal(0, 20, (H, W, 3)).astype(np.float32)
    assert np.allclose(O.gradient_magnitude(lab.transpose(1, 0, 2)), O.gradient_magnitude(lab).T,
                       rtol=0, atol=1e-12)
    # mirroring x keeps every magnitude (the differences change sign only)
    assert np.allclose(O.gradient_magnitude(lab[:, ::-1]), O.gradient_magnitude(lab)[:, ::-1],
                       rtol=0, atol=1e-12)


def test_contour_constant_and_range():
    assert (O.contour_prior(np.full((5, 6, 3), 42.0, np.float32)) == 0).all()
    assert (O.contour_prior(np.zeros((1, 1, 3), np.float32)) == 0).all()
    rng = np.random.default_rng(3)
    c = O.contour_prior(rng.uniform(-50, 50, (30, 40, 3)).astype(np.float32))
    assert c.dtype == np.float32 and c.min() >= 0 and c.max() == 1.0
