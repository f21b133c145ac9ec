"""Pins for the oracle's window form of the assignment (the candidate rule of
Algorithm 1: the candidates of a pixel are the clusters whose (2r+1) x (2r+1)
window around the barycenter contains it; the smallest D wins, the smallest k
among equal D, and pixels no window contains keep their label)."""
import numpy as np
import pytest

from test_oracle_assign import _brute_f32, _random_state

F32 = np.float32


def _window_brute(orc, g, lab, w, c, e, prev, R, lam, gamma, spw):
    H, W = g.height, g.width
    out = prev.copy()
    best = np.full((H, W), np.inf, F32)
    centre = [(int(np.floor(F32(c[k, 3]) + F32(0.5))), int(np.floor(F32(c[k, 4]) + F32(0.5))))
              for k in range(g.num_sp)]
    for y in range(H):
        for x in range(W):
            for k in range(g.num_sp):                      # ascending k, strict '<'
                cx = min(max(centre[k][0], 0), W - 1)
                cy = min(max(centre[k][1], 0), H - 1)
                if abs(x - cx) > R or abs(y - cy) > R:
                    continue
                d = _brute_f32(lab, w, x, y, c[k], e[k], lam, gamma, spw)
                if d < best[y, x]:
                    best[y, x] = d
                    out[y, x] = k
    return out, best


@pytest.mark.parametrize("W,H,k,R,seed", [(19, 13, 6, None, 1), (24, 20, 12, 2, 2), (17, 23, 4, 5, 3),
                                          (16, 16, 16, 0, 4)])
def test_window_assignment_brute_force(orc, W, H, k, R, seed):
    lab, con, g, c, e = _random_state(orc, W, H, k, seed, jitter=2.5)
    w = orc.wmap(con)
    gamma, spw = orc.default_gamma(g), orc.spatial_weight(g)
    if R is None:
        R = orc.window_radius(g)
    prev = np.random.default_rng(seed).integers(0, g.num_sp, (H, W)).astype(np.int32)
    got, best = orc.assign_window(g, lab, w, c, e, prev, gamma=gamma, spw=spw, R=R)
    ref, ref_best = _window_brute(orc, g, lab, w, c, e, prev, R, 0.5, gamma, spw)
    assert (got == ref).all()
    assert (best == ref_best).all()
    if R == 0:
        # a zero-radius window covers only the rounded barycenter itself
        assert (got != prev).sum() <= g.num_sp


def test_window_radius_is_rounded_grid_step(orc):
    assert orc.window_radius(orc.grid(1920, 1080, 2000)) == 32     # r = 32.2
    assert orc.window_radius(orc.grid(481, 321, 250)) == 25        # r = 24.85
    assert orc.window_radius(orc.grid(64, 48, 12)) == 16           # r = 16


def test_window_run_constant_image_fixed_point(orc):
    """On a constant image with no contours the cell grid is a fixed point of the
    window form too (every pixel is covered by its own cell's window)."""
    W, H, k = 64, 48, 12
    lab = np.full((H, W, 3), [30.0, 5.0, -5.0], F32)
    con = np.zeros((H, W), F32)
    g = orc.grid(W, H, k)
    c0, e0, l0 = orc.init_grid(g, lab)
    r = orc.run_window(lab, con, k, iterations=5)
    assert (r.labels == l0).all() and (r.centres == c0).all()


def test_window_transpose_equivariance(orc):
    W, H, k = 52, 37, 12
    lab, con, g, c, e = _random_state(orc, W, H, k, 9)
    w = orc.wmap(con)
    prev = np.zeros((H, W), np.int32)
    lbl, best = orc.assign_window(g, lab, w, c, e, prev)
    gt = orc.grid(H, W, k)
    perm = np.empty(g.num_sp, np.int64)
    for i in range(g.ny):
        for j in range(g.nx):
            perm[i * g.nx + j] = j * gt.nx + i
    ct = np.empty_like(c)
    ct[perm] = c[:, [0, 1, 2, 4, 3]]
    et = np.empty_like(e)
    et[perm] = e[:, ::-1]
    # ties cannot occur on random data, so the visiting order of clusters does not matter
    lt, bt = orc.assign_window(gt, np.ascontiguousarray(lab.transpose(1, 0, 2)),
                               np.ascontiguousarray(w.T), ct, et, prev.T.copy())
    assert (bt.T == best).all()
    covered = np.isfinite(best)
    assert (lt.T[covered] == perm[lbl[covered]]).all()


def test_window_ties_go_to_lowest_k(orc):
    """Identical clusters: every covered pixel sees equal distances and keeps the
    first (lowest) k; uncovered pixels keep their previous label."""
    W, H, k = 40, 30, 6
    g = orc.grid(W, H, k)
    lab = np.full((H, W, 3), 20.0, F32)
    w = np.zeros((H, W), F32)
    c = np.tile(np.array([20.0, 0.0, 0.0, 18.0, 12.0], F32), (g.num_sp, 1))
    e = np.tile(np.array([18, 12], np.int32), (g.num_sp, 1))
    prev = np.full((H, W), 5, np.int32)
    R = 4
    got, best = orc.assign_window(g, lab, w, c, e, prev, R=R)
    inside = np.zeros((H, W), bool)
    inside[12 - R:12 + R + 1, 18 - R:18 + R + 1] = True
    assert (got[inside] == 0).all() and (got[~inside] == 5).all()
    assert np.isinf(best[~inside]).all()
