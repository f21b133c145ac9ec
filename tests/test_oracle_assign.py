"""Pins for the oracle's distance (Eqs. (1)-(3)) and assignment (Algorithm 1).

  * worked examples whose value is derived by hand (dyadic inputs, so the
    FP32 result is exact);
  * the SLIC special case (lambda = 1, gamma = 0 reduce Eq. (3) to the SLIC
    distance, Sec. II-D) against a vectorised textbook 3x3 SLIC assignment;
  * an independent brute-force evaluator: paths from exact rational
    nearest-integer rounding, the distance in FP32 scalars (bit-exact), and
    in FP64 over ALL clusters (the chosen label must be the FP64 argmin among
    the grid neighbours up to FP32 rounding);
  * equivariance under transposing the image plane (catches swapped x/y);
  * a constant image is a fixed point of the grid; a contour wall has no
    effect where the colour distance is zero and a predictable one elsewhere.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_1903_07149_amd import synth

F32 = np.float32


def test_worked_example_row(orc):
    # 4x1 row, p = (0,0), endpoint (3,0): the path is all four pixels.
    # L = 4, 2, 0, 0 (a = b = 0), centre colour 0: d_c = 16, 4, 0, 0, sum 20, |P| = 4.
    # lambda = 0.5: A = 0.5*16 + 0.5*(20/4) = 10.5.
    # w = 0, 0.5, 0.25, 0: sum 0.75; gamma = 4: B = 1 + 4*(0.75/4) = 1.75.
    # X_k = (3, 0): d_s = 9; m^2/r^2 = 0.5: D = 10.5*1.75 + 9*0.5 = 22.875.
    lab = np.zeros((1, 4, 3), F32)
    lab[0, :, 0] = [4, 2, 0, 0]
    w = np.array([[0, 0.5, 0.25, 0]], F32)
    d = orc.distance(lab, w, 0, 0, [0, 0, 0, 3.0, 0.0], (3, 0), lam=0.5, gamma=4.0, spw=0.5)
    assert d == 22.875


def test_worked_example_diagonal(orc):
    # 3x2 image, p = (0,0), X_k = (2.25, 0.75) -> endpoint (2,1); path (0,0),(1,1),(2,1).
    # centre colour (1, 2, -1).  f(0,0) = (1,4,-1): d_c = 4; f(1,1) = (3,2,1): d_c = 8;
    # f(2,1) = (1,2,-1): d_c = 0.  lambda = 0.25: A = 0.25*4 + 0.75*(12/3) = 4.
    # w = 0.5, 1, 0 on the path: B = 1 + 2*(1.5/3) = 2.
    # d_s = 2.25^2 + 0.75^2 = 5.625, m^2/r^2 = 0.25: D = 8 + 1.40625 = 9.40625.
    lab = np.zeros((2, 3, 3), F32)
    lab[0, 0] = [1, 4, -1]
    lab[1, 1] = [3, 2, 1]
    lab[1, 2] = [1, 2, -1]
    lab[0, 1] = [50, 50, 50]      # off-path pixels must not matter
    lab[0, 2] = [-50, 9, 9]
    lab[1, 0] = [7, 7, 7]
    w = np.array([[0.5, 0.9, 0.9], [0.9, 1.0, 0.0]], F32)
    d = orc.distance(lab, w, 0, 0, [1, 2, -1, 2.25, 0.75], (2, 1), lam=0.25, gamma=2.0, spw=0.25)
    assert d == 9.40625


def _candidates(g, x, y):
    ci = y * g.ny // g.height
    cj = x * g.nx // g.width
    out = []
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            ii, jj = ci + di, cj + dj
            if 0 <= ii < g.ny and 0 <= jj < g.nx:
                out.append(ii * g.nx + jj)
    return out


def _random_state(orc, W, H, k, seed, jitter=3.0):
    """Random image and a perturbed grid state (centres moved, endpoints rounded)."""
    lab, contour = synth.random_lab(W, H, seed)
    g = orc.grid(W, H, k)
    centres, ep, _ = orc.init_grid(g, lab)
    rng = np.random.default_rng(seed + 100)
    centres = centres.copy()
    centres[:, 0:3] += rng.normal(0, 10, (g.num_sp, 3)).astype(F32)
    centres[:, 3] = np.clip(centres[:, 3] + rng.uniform(-jitter, jitter, g.num_sp), 0, W - 1)
    centres[:, 4] = np.clip(centres[:, 4] + rng.uniform(-jitter, jitter, g.num_sp), 0, H - 1)
    ep = orc.round_endpoints(g, centres)
    return lab, contour, g, centres.astype(F32), ep


def test_slic_special_case(orc):
    """lambda = 1, gamma = 0: D = d_c + d_s m^2/r^2, the SLIC distance (Sec. II-D)."""
    for seed, (W, H, k) in enumerate([(61, 47, 30), (128, 96, 48), (37, 90, 12)]):
        lab, contour, g, centres, ep = _random_state(orc, W, H, k, seed)
        w = orc.wmap(contour)
        spw = F32(orc.spatial_weight(g))
        labels, _, _ = orc.assign(g, lab, w, centres, ep, lam=1.0, gamma=0.0, spw=float(spw))
        # vectorised textbook SLIC over the 3x3 grid neighbours
        yy, xx = np.mgrid[0:H, 0:W]
        ci = yy * g.ny // H
        cj = xx * g.nx // W
        best = np.full((H, W), np.inf, F32)
        lbl = np.full((H, W), -1, np.int64)
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                ii, jj = ci + di, cj + dj
                ok = (ii >= 0) & (ii < g.ny) & (jj >= 0) & (jj < g.nx)
                kk = np.where(ok, ii * g.nx + jj, 0)
                c = centres[kk]
                dl = lab[..., 0] - c[..., 0]
                da = lab[..., 1] - c[..., 1]
                db = lab[..., 2] - c[..., 2]
                dcol = (dl * dl + da * da) + db * db
                ex = xx.astype(F32) - c[..., 3]
                ey = yy.astype(F32) - c[..., 4]
                D = dcol + (ex * ex + ey * ey) * spw
                D = np.where(ok, D, np.inf).astype(F32)
                take = D < best
                best = np.where(take, D, best)
                lbl = np.where(take, kk, lbl)
        assert (labels == lbl).all()


def _rational_path(x0, y0, x1, y1):
    dx, dy = x1 - x0, y1 - y0
    n = max(abs(dx), abs(dy))
    pts = []
    for i in range(n + 1):
        out = []
        for a0, d in ((x0, dx), (y0, dy)):
            v = Fraction(a0) + (Fraction(i * d, n) if n else 0)
            fl = v.numerator // v.denominator
            fr = v - fl
            out.append(fl + 1 if fr > Fraction(1, 2) or (fr == Fraction(1, 2) and d > 0) else fl)
        pts.append(tuple(out))
    return pts


def _brute_f32(lab, w, x, y, c, e, lam, gamma, spw):
    lam, gamma, spw = F32(lam), F32(gamma), F32(spw)
    sc = F32(0)
    sw = F32(0)
    path = _rational_path(x, y, int(e[0]), int(e[1]))
    for (qx, qy) in path:
        f = lab[qy, qx]
        dl, da, db = f[0] - c[0], f[1] - c[1], f[2] - c[2]
        sc = F32(sc + F32(F32(F32(dl * dl) + F32(da * da)) + F32(db * db)))
        sw = F32(sw + w[qy, qx])
    f = lab[y, x]
    dl, da, db = f[0] - c[0], f[1] - c[1], f[2] - c[2]
    dcp = F32(F32(F32(dl * dl) + F32(da * da)) + F32(db * db))
    npf = F32(len(path))
    A = F32(F32(lam * dcp) + F32(F32(F32(1) - lam) * F32(sc / npf)))
    B = F32(F32(1) + F32(gamma * F32(sw / npf)))
    ex = F32(F32(x) - c[3])
    ey = F32(F32(y) - c[4])
    return F32(F32(A * B) + F32(F32(F32(ex * ex) + F32(ey * ey)) * spw))


def _brute_f64(lab, w, x, y, c, e, lam, gamma, spw):
    path = _rational_path(x, y, int(e[0]), int(e[1]))
    cc = np.asarray(c, np.float64)
    fq = np.array([lab[qy, qx] for qx, qy in path], np.float64)
    wq = np.array([w[qy, qx] for qx, qy in path], np.float64)
    dq = ((fq - cc[:3]) ** 2).sum(axis=1)
    dcp = ((lab[y, x].astype(np.float64) - cc[:3]) ** 2).sum()
    A = lam * dcp + (1 - lam) * dq.mean()
    B = 1 + gamma * wq.mean()
    return A * B + ((x - cc[3]) ** 2 + (y - cc[4]) ** 2) * spw


@pytest.mark.parametrize("W,H,k,lam,seed", [(13, 9, 6, 0.5, 1), (24, 16, 8, 0.5, 2),
                                            (17, 23, 9, 0.0, 3), (20, 20, 16, 0.8, 4)])
def test_brute_force_tiny(orc, W, H, k, lam, seed):
    lab, contour, g, centres, ep = _random_state(orc, W, H, k, seed, jitter=4.0)
    w = orc.wmap(contour)
    gamma = orc.default_gamma(g)
    spw = orc.spatial_weight(g)
    labels, best, _ = orc.assign(g, lab, w, centres, ep, lam=lam, gamma=gamma, spw=spw)
    for y in range(H):
        for x in range(W):
            cands = _candidates(g, x, y)
            d32 = [_brute_f32(lab, w, x, y, centres[kk], ep[kk], lam, gamma, spw) for kk in cands]
            i32 = int(np.argmin(d32))                    # first minimum = strict '<' in k order
            assert labels[y, x] == cands[i32]
            assert best[y, x] == d32[i32]
            # FP64 over all clusters: the grid-neighbour argmin is the label up to rounding
            d64 = {kk: _brute_f64(lab, w, x, y, centres[kk], ep[kk], lam, gamma, spw)
                   for kk in range(g.num_sp)}
            near = min(d64[kk] for kk in cands)
            assert d64[int(labels[y, x])] <= near * (1 + 1e-5) + 1e-4
            assert abs(float(best[y, x]) - d64[int(labels[y, x])]) <= 1e-5 * near + 1e-4


def test_transpose_equivariance(orc):
    W, H, k = 70, 45, 24
    lab, contour, g, centres, ep = _random_state(orc, W, H, k, 11)
    w = orc.wmap(contour)
    labels, best, _ = orc.assign(g, lab, w, centres, ep, gamma=orc.default_gamma(g),
                                 spw=orc.spatial_weight(g))
    gt = orc.grid(H, W, k)
    assert (gt.nx, gt.ny) == (g.ny, g.nx)
    # cluster (i, j) of the original grid is (j, i) of the transposed one
    perm = np.empty(g.num_sp, np.int64)
    for i in range(g.ny):
        for j in range(g.nx):
            perm[i * g.nx + j] = j * gt.nx + i
    ct = np.empty_like(centres)
    ct[perm] = centres[:, [0, 1, 2, 4, 3]]
    et = np.empty_like(ep)
    et[perm] = ep[:, ::-1]
    lt, bt, _ = orc.assign(gt, np.ascontiguousarray(lab.transpose(1, 0, 2)), np.ascontiguousarray(w.T),
                           ct, et, gamma=orc.default_gamma(gt), spw=orc.spatial_weight(gt))
    assert (lt.T == perm[labels]).all()
    assert (bt.T == best).all()


def test_constant_image_fixed_point(orc):
    W, H, k = 64, 48, 12            # r = 16, 4 x 3 cells of 16 x 16
    lab = np.empty((H, W, 3), F32)
    lab[...] = [55.0, -3.0, 12.0]
    contour = np.zeros((H, W), F32)
    g = orc.grid(W, H, k)
    assert (g.nx, g.ny) == (4, 3)
    c0, e0, l0 = orc.init_grid(g, lab)
    r = orc.run(lab, contour, k, iterations=10)
    assert (r.labels == l0).all()
    assert (r.centres == c0).all() and (r.endpoints == e0).all()
    assert (r.counts == 256).all()


def test_contour_wall_needs_colour_difference(orc):
    """A contour wall on a constant-colour image changes nothing: d_C multiplies d_c (Eq. 3)."""
    W, H, k = 40, 20, 2
    lab = np.full((H, W, 3), 40.0, F32)
    wall = np.zeros((H, W), F32)
    wall[:, 12] = 1.0
    r0 = orc.run(lab, np.zeros((H, W), F32), k, iterations=3)
    r1 = orc.run(lab, wall, k, iterations=3)
    assert (r0.labels == r1.labels).all()


def test_contour_wall_moves_boundary(orc):
    """Two clusters on a noisy flat image split at x = 20; a wall at x = 14 with a slight
    colour step there pulls the boundary onto the wall, exactly as the FP64 brute force says."""
    W, H, k = 40, 20, 2
    rng = np.random.default_rng(3)
    lab = (np.full((H, W, 3), 40.0) + rng.normal(0, 0.5, (H, W, 3))).astype(F32)
    lab[:, 14:, 0] += 6.0
    wall = np.zeros((H, W), F32)
    wall[:, 14] = 1.0
    g = orc.grid(W, H, k)
    assert (g.nx, g.ny) == (2, 1)
    c, e, _ = orc.init_grid(g, lab)
    w = orc.wmap(wall)
    gamma = orc.default_gamma(g)
    spw = orc.spatial_weight(g)
    labels, _, _ = orc.assign(g, lab, w, c, e, gamma=gamma, spw=spw)
    for y in range(H):
        for x in range(W):
            d = [_brute_f64(lab, w, x, y, c[kk], e[kk], 0.5, gamma, spw) for kk in range(2)]
            if abs(d[0] - d[1]) > 1e-4 * max(d):
                assert labels[y, x] == int(np.argmin(d))
    nowall, _, _ = orc.assign(g, lab, orc.wmap(np.zeros_like(wall)), c, e, gamma=gamma, spw=spw)
    # the wall moves pixels between x = 14 and the old boundary to the right cluster
    moved = (labels != nowall)
    assert moved.any()
    xs = np.nonzero(moved)[1]
    assert xs.min() >= 14 and xs.max() < 20


def test_thread_count_independent(orc):
    img = synth.make_image(160, 120, 12, 10.0, 5)
    orc.set_threads(1)
    a = orc.run(img.lab, img.contour, 60, iterations=3)
    orc.set_threads(orc.max_threads() if orc.max_threads() > 1 else 4)
    orc.set_threads(4)
    b = orc.run(img.lab, img.contour, 60, iterations=3)
    assert (a.labels == b.labels).all() and (a.centres == b.centres).all()
    assert a.samples == b.samples


def test_ties_go_to_lowest_k(orc):
    """Identical clusters give identical D everywhere; strict '<' over ascending k keeps
    the first candidate (Algorithm 1), so every pixel takes its lowest-index neighbour."""
    W, H, k = 48, 32, 6
    g = orc.grid(W, H, k)
    assert (g.nx, g.ny) == (3, 2)
    lab = np.full((H, W, 3), 20.0, F32)
    w = np.zeros((H, W), F32)
    centres = np.tile(np.array([20.0, 0.0, 0.0, 23.0, 15.0], F32), (g.num_sp, 1))
    ep = np.tile(np.array([23, 15], np.int32), (g.num_sp, 1))
    labels, _, _ = orc.assign(g, lab, w, centres, ep, gamma=orc.default_gamma(g),
                              spw=orc.spatial_weight(g))
    yy, xx = np.mgrid[0:H, 0:W]
    ci, cj = yy * g.ny // H, xx * g.nx // W
    lowest = np.maximum(ci - 1, 0) * g.nx + np.maximum(cj - 1, 0)
    assert (labels == lowest).all()
