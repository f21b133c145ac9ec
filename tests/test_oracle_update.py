"""Pins for the oracle's update (Algorithm 1: mean colour and barycenter of
each superpixel), projection (Sec. II-D Remark, Eq. (4)) and whole runs."""
from fractions import Fraction

import numpy as np
import pytest

from paper_1903_07149_amd import synth

F32 = np.float32


def _numpy_means(lab, labels, K):
    H, W = labels.shape
    lbl = labels.ravel()
    cnt = np.bincount(lbl, minlength=K).astype(np.float64)
    yy, xx = np.mgrid[0:H, 0:W]
    out = np.zeros((K, 5), np.float64)
    for ch in range(3):
        out[:, ch] = np.bincount(lbl, weights=lab[..., ch].ravel().astype(np.float64), minlength=K)
    out[:, 3] = np.bincount(lbl, weights=xx.ravel().astype(np.float64), minlength=K)
    out[:, 4] = np.bincount(lbl, weights=yy.ravel().astype(np.float64), minlength=K)
    nz = cnt > 0
    out[nz] /= cnt[nz, None]
    return out, cnt.astype(np.int64)


def test_update_matches_library_means(orc):
    img = synth.make_image(97, 73, 9, 10.0, 21)
    g = orc.grid(97, 73, 30)
    rng = np.random.default_rng(0)
    labels = rng.integers(0, g.num_sp, (73, 97)).astype(np.int32)
    labels[labels == 5] = 6                          # superpixel 5 is empty
    prev = rng.normal(0, 1, (g.num_sp, 5)).astype(F32)
    new, counts = orc.update(g, img.lab, labels, prev)
    ref, cnt = _numpy_means(img.lab, labels, g.num_sp)
    assert (counts == cnt).all() and counts.sum() == 97 * 73
    nz = cnt > 0
    assert (new[nz] == ref[nz].astype(F32)).all()     # same FP64 raster sums, one rounding
    assert (new[~nz] == prev[~nz]).all()              # empty superpixel keeps its centre


def test_fixed_point_mean_is_exact_mean_rounded(orc):
    img = synth.make_image(40, 30, 4, 10.0, 3)
    g = orc.grid(40, 30, 12)
    rng = np.random.default_rng(1)
    labels = rng.integers(0, g.num_sp, (30, 40)).astype(np.int32)
    fixed, _ = orc.update(g, img.lab, labels, np.zeros((g.num_sp, 5), F32), mode=orc.MEAN_FIXED)
    plain, _ = orc.update(g, img.lab, labels, np.zeros((g.num_sp, 5), F32))
    for k in range(g.num_sp):
        vals = img.lab.reshape(-1, 3)[labels.ravel() == k]
        for ch in range(3):
            exact = sum((Fraction(float(v)) for v in vals[:, ch]), Fraction(0)) / len(vals)
            # fixed-point quantisation is 2^-25 per pixel, so the mean is within 2^-25 + 1 ulp
            tol = 2.0 ** -25 + float(np.spacing(F32(abs(float(exact)))))
            assert abs(float(fixed[k, ch]) - float(exact)) <= tol
            assert abs(float(plain[k, ch]) - float(exact)) <= float(np.spacing(F32(abs(float(exact)))))
    assert (fixed[:, 3:] == plain[:, 3:]).all()       # integer position sums: exact either way


def test_update_idempotent(orc):
    img = synth.make_image(64, 64, 6, 10.0, 4)
    r = orc.run(img.lab, img.contour, 16, iterations=3)
    g = orc.grid(64, 64, 16)
    c1, n1 = orc.update(g, img.lab, r.labels, r.centres)
    c2, n2 = orc.update(g, img.lab, r.labels, c1)
    assert (c1 == c2).all() and (n1 == n2).all()


def test_projection_c_shape(orc):
    """A C-shaped superpixel whose barycenter is outside it: Eq. (4) by brute force."""
    W, H = 30, 30
    g = orc.grid(W, H, 4)                              # 2 x 2 grid, k = 0..3
    labels = np.ones((H, W), np.int32)
    cshape = np.zeros((H, W), bool)
    cshape[5:25, 5:9] = True
    cshape[5:9, 5:22] = True
    cshape[21:25, 5:22] = True
    labels[cshape] = 0
    lab = np.zeros((H, W, 3), F32)
    centres, counts = orc.update(g, lab, labels, np.zeros((4, 5), F32))
    ep0 = orc.round_endpoints(g, centres)
    assert labels[ep0[0, 1], ep0[0, 0]] != 0          # barycenter falls in the hollow
    ep, moved = orc.project(g, labels, centres, counts, ep0)
    ys, xs = np.nonzero(labels == 0)
    d = (xs.astype(F32) - centres[0, 3]) ** 2 + (ys.astype(F32) - centres[0, 4]) ** 2
    order = np.lexsort((ys * W + xs, d))               # by distance, then raster index
    assert tuple(ep[0]) == (xs[order[0]], ys[order[0]])
    assert labels[ep[0, 1], ep[0, 0]] == 0
    assert moved >= 1
    # superpixels 2 and 3 are empty: endpoints untouched
    assert (ep[2:] == ep0[2:]).all()


def test_init_grid_cells(orc):
    W, H, k = 481, 321, 250
    g = orc.grid(W, H, k)
    assert (g.nx, g.ny, g.num_sp) == (19, 13, 247)
    lab = synth.random_lab(W, H, 0)[0]
    c, e, labels = orc.init_grid(g, lab)
    yy, xx = np.mgrid[0:H, 0:W]
    assert (labels == (yy * g.ny // H) * g.nx + xx * g.nx // W).all()
    ref, cnt = _numpy_means(lab, labels, g.num_sp)
    assert (c == ref.astype(F32)).all()
    assert (e[:, 0] == np.floor(c[:, 3] + F32(0.5))).all()
    # cell sizes differ by at most one row / column
    assert cnt.max() - cnt.min() <= 26 + 25 + 1


@pytest.mark.parametrize("wl", [synth.BSD_SHAPE])
def test_run_invariants(orc, wl):
    img = synth.workload_image(wl)
    H, W = img.contour.shape
    r = orc.run(img.lab, img.contour, wl.k, iterations=wl.iterations)
    g = orc.grid(W, H, wl.k)
    K = g.num_sp
    assert r.labels.min() >= 0 and r.labels.max() < K
    assert r.counts.sum() == W * H
    # every label is a grid neighbour of the pixel's own cell
    yy, xx = np.mgrid[0:H, 0:W]
    ci, cj = yy * g.ny // H, xx * g.nx // W
    li, lj = r.labels // g.nx, r.labels % g.nx
    assert (np.abs(li - ci) <= 1).all() and (np.abs(lj - cj) <= 1).all()
    nz = r.counts > 0
    # after projection every non-empty superpixel contains its endpoint
    assert (r.labels[r.endpoints[nz, 1], r.endpoints[nz, 0]] == np.nonzero(nz)[0]).all()
    # barycenters lie in the bounding box of their pixels
    for k in np.nonzero(nz)[0][::7]:
        ys, xs = np.nonzero(r.labels == k)
        assert xs.min() <= r.centres[k, 3] <= xs.max() and ys.min() <= r.centres[k, 4] <= ys.max()
    # the final centres are the update of the final labels
    c, n = orc.update(g, img.lab, r.labels, r.centres)
    assert (c == r.centres).all() and (n == r.counts).all()
    # reading: the paper sets 5 iterations; the runs here use 10, and stop nowhere early
    assert r.samples > 0


def test_resume_is_exact(orc):
    """The state between iterations is (centres, endpoints): run(4) == run(2) then 2 more."""
    img = synth.make_image(120, 90, 10, 10.0, 8)
    g = orc.grid(120, 90, 40)
    full = orc.run(img.lab, img.contour, 40, iterations=4)
    half = orc.run(img.lab, img.contour, 40, iterations=2)
    w = orc.wmap(img.contour)
    c, e = half.centres, half.endpoints
    for _ in range(2):
        lbl, _, _ = orc.assign(g, img.lab, w, c, e, gamma=orc.default_gamma(g),
                               spw=orc.spatial_weight(g))
        c, n = orc.update(g, img.lab, lbl, c)
        e, _ = orc.project(g, lbl, c, n, e)
    assert (lbl == full.labels).all() and (c == full.centres).all() and (e == full.endpoints).all()
