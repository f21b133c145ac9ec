"""Pins for the FP64 soft-SCALP oracle (an extension: softmax over the
distances of Eq. (3) with temperature T, soft barycenter update).

  * its analytic gradient against FP64 central finite differences of its own
    forward (eps = 1e-4) on 32x32 crops with K = 16;
  * T -> 0: the argmax of Q is the hard assignment of Algorithm 1, and a
    one-hot Q makes the soft update equal to the hard update.
"""
import numpy as np
import pytest

from paper_1903_07149_amd import synth


def _crop_batch(n, size=32, seed=500):
    labs, cons = [], []
    for b in range(n):
        img = synth.make_image(size, size, 6, 10.0, seed + b)
        labs.append(img.lab)
        cons.append(img.contour)
    return np.stack(labs), np.stack(cons)


def _loss(orc, lab, con, k, gq, gth, iters, T):
    th, q, _ = orc.soft_forward(lab, con, k, iterations=iters, T=T)
    return float((gq * q[-1]).sum() + (gth * th[-1]).sum()), th


@pytest.mark.parametrize("T,iters", [(50.0, 2), (0.5, 2), (5.0, 3)])
def test_soft_gradient_finite_differences(orc, T, iters):
    k = 16
    lab, con = _crop_batch(1)
    # soft contour values so that dw/dC is not ~0 everywhere
    con = np.clip(con + 0.15 * np.random.default_rng(1).random(con.shape), 0, 1).astype(np.float32)
    g = orc.grid(32, 32, k)
    rng = np.random.default_rng(2)
    gq = rng.normal(0, 1, (1, 32, 32, 9))
    gth = rng.normal(0, 1, (1, g.num_sp, 5))
    glab, gcon = orc.soft_backward(lab, con, k, gq, gth, iterations=iters, T=T)
    eps = 1e-4
    checked = 0
    idx_lab = [tuple(rng.integers(0, s) for s in lab.shape) for _ in range(40)]
    idx_con = [tuple(rng.integers(0, s) for s in con.shape) for _ in range(25)]
    for arr, grad, idxs in ((lab, glab, idx_lab), (con, gcon, idx_con)):
        for idx in idxs:
            base = arr[idx]
            if arr is con and (base - eps < 0 or base + eps > 1):
                continue
            vals = []
            eps_ok = True
            ends = []
            for s in (+1, -1):
                a = arr.copy()
                # FD in FP64 on an FP32 input: the step is applied in FP64 through the value
                a = a.astype(np.float64)
                a[idx] = base + s * eps
                a32 = a.astype(np.float32)
                # the oracle consumes FP32 inputs; use an exactly representable step
                h = float(a32[idx]) - float(base)
                if h == 0.0:
                    eps_ok = False
                    break
                args = (a32, con, k) if arr is lab else (lab, a32, k)
                L, th = _loss(orc, *args, gq, gth, iters, T)
                vals.append((L, h))
                ends.append(np.floor(th[:-1, ..., 3:5] + 0.5))
            if not eps_ok or not (ends[0] == ends[1]).all():
                continue                              # an endpoint rounding flipped: FD invalid
            (lp, hp), (lm, hm) = vals
            fd = (lp - lm) / (hp - hm)
            an = float(grad[idx])
            assert abs(fd - an) <= 2e-3 * max(1.0, abs(an)) + 2e-3 * abs(fd), (idx, fd, an)
            checked += 1
    assert checked >= 40


def test_soft_zero_temperature_is_hard(orc):
    """Integer Lab on 4x4-pixel cells: the FP32 hard and FP64 soft initial centres coincide,
    so argmax Q at T -> 0 is the hard assignment and a one-hot Q gives the hard update."""
    W = H = 16
    k = 16
    rng = np.random.default_rng(4)
    lab = rng.integers(0, 60, (H, W, 3)).astype(np.float32)
    con = (rng.integers(0, 5, (H, W)) / 4.0).astype(np.float32)
    g = orc.grid(W, H, k)
    assert (g.nx, g.ny) == (4, 4)
    th, q, z = orc.soft_forward(lab[None], con[None], k, iterations=1, T=1e-4)
    c0, e0, _ = orc.init_grid(g, lab)
    assert (th[0, 0] == c0.astype(np.float64)).all()
    hard, _, _ = orc.assign(g, lab, orc.wmap(con), c0, e0, gamma=orc.default_gamma(g),
                            spw=orc.spatial_weight(g))
    yy, xx = np.mgrid[0:H, 0:W]
    ci, cj = yy * g.ny // H, xx * g.nx // W
    j = q[0, 0].argmax(axis=-1)
    soft_lbl = (ci + j // 3 - 1) * g.nx + (cj + j % 3 - 1)
    assert (soft_lbl == hard).all()
    assert np.allclose(q[0, 0].max(axis=-1), 1.0)
    onehot = (q[0, 0].max(axis=-1) == 1.0)
    if onehot.all():
        c1, n1 = orc.update(g, lab, hard, c0)
        nz = n1 > 0
        assert (th[1, 0][nz] .astype(np.float32) == c1[nz]).all()
        assert (z[0, 0][nz] == n1[nz]).all()


def test_soft_forward_shapes_and_simplex(orc):
    lab, con = _crop_batch(2)
    th, q, z = orc.soft_forward(lab, con, 16, iterations=3, T=0.5)
    assert th.shape == (4, 2, 16, 5) and q.shape == (3, 2, 32, 32, 9) and z.shape == (3, 2, 16)
    assert np.allclose(q.sum(-1), 1.0) and (q >= 0).all()
    assert np.allclose(z.sum(-1), 32 * 32)
    # corner pixels see only 4 of the 9 neighbours
    assert (q[:, :, 0, 0, [0, 1, 2, 3, 6]] == 0).all()


def test_d32_mode_matches_fp64_and_hard(orc):
    """The FP32-distance mode agrees with the all-FP64 mode to FP32 accuracy where
    the problem is well conditioned (T = 50), and its first soft step at T -> 0 is
    exactly the hard oracle's assignment."""
    lab, con = _crop_batch(2)
    k = 16
    th64, q64, _ = orc.soft_forward(lab, con, k, iterations=2, T=50.0)
    th32, q32, _ = orc.soft_forward(lab, con, k, iterations=2, T=50.0, d32=True)
    assert np.abs(q64 - q32).max() < 1e-4
    assert (np.abs(th64 - th32) / (np.abs(th64) + 1)).max() < 1e-4
    assert (th32 == th32.astype(np.float32)).all() and (q32 == q32.astype(np.float32)).all()
    g = orc.grid(32, 32, k)
    rng = np.random.default_rng(3)
    gq = rng.normal(0, 1, (2, 32, 32, 9))
    gth = rng.normal(0, 1, (2, g.num_sp, 5))
    a64 = orc.soft_backward(lab, con, k, gq, gth, iterations=2, T=50.0)
    a32 = orc.soft_backward(lab, con, k, gq, gth, iterations=2, T=50.0, d32=True)
    for x, y in zip(a64, a32):
        assert np.linalg.norm(x - y) / np.linalg.norm(x) < 1e-3
    # T -> 0 (FP64 exp underflows: Q is exactly one-hot) on the hard oracle's state
    th, q, _ = orc.soft_forward(lab[:1], con[:1], k, iterations=1, T=1e-6, d32=True)
    c0, e0, _ = orc.init_grid(g, lab[0])
    assert (th[0, 0].astype(np.float32) == c0).all()
    hard, _, _ = orc.assign(g, lab[0], orc.wmap(con[0]), c0, e0)
    yy, xx = np.mgrid[0:32, 0:32]
    j = q[0, 0].argmax(axis=-1)
    lbl = (yy * g.ny // 32 + j // 3 - 1) * g.nx + (xx * g.nx // 32 + j % 3 - 1)
    assert (lbl == hard).all()


def test_tiny_mass_keeps_centre(orc):
    """A superpixel whose soft mass falls below 1e-6 keeps its previous centre."""
    W = H = 32                                     # 4 x 4 cells of 8 x 8
    lab = np.full((H, W, 3), [50.0, 60.0, -60.0], np.float32)
    lab[:, :12] = [50.0, -60.0, 60.0]              # colour edge through the middle of column 1
    con = np.zeros((H, W), np.float32)
    for d32 in (False, True):
        th, q, z = orc.soft_forward(lab[None], con[None], 16, iterations=2, T=0.05, d32=d32)
        # the cells of column 1 average both colours: every pixel is far closer to a pure
        # neighbour, so their soft mass vanishes and they keep their centres
        light = z[0, 0] < 1e-6
        assert light.sum() == 4 and light.reshape(4, 4)[:, 1].all()
        assert (th[1, 0][light] == th[0, 0][light]).all()
        assert (z[0, 0][~light] > 1.0).all()
