"""Soft SCALP on the GPU against the oracle's FP32-distance mode (d32: the same
FP32 distance as the hard path, FP64 softmax and update sums, Q and Theta
rounded to FP32 where produced).

Tolerances: both sides compute bit-identical FP32 distances, so Q differs only
where the two FP64 exponentials (each within 1 ulp) round to different FP32
values: |dQ| <= 1e-6.  Theta differs only by the order of its FP64 sums
before the single FP32 rounding: relative 1e-6.

Gradients are compared element by element with the oracle run with the same
Q < 2^-24 cut as the GPU backward (the cut itself is pinned against the plain
chain rule on the CPU, tests/test_oracle_soft_bound.py, and here once more at
a temperature where many Q sit near the cut): |got - ref| <= 2^-24 E + Md per
element, E being the oracle's running error bound of an FP32 evaluation of
the backward (first order; dL/dTheta taken as FP64 sums of FP32 partials no
longer than one path, which is how the GPU sums it) and Md what the slots
whose Q lies within one ulp of the cut can change.  The relative L2 error of
the whole gradient (<= 1e-3) is checked as well.
"""
import os

import numpy as np
import pytest

from paper_1903_07149_amd import synth
from gpu_util import dev, host, needs_gpu, say, torch

pytestmark = [pytest.mark.gpu, needs_gpu]


def _batch(B, size, regions, seed0, k=None):
    labs, cons = [], []
    for b in range(B):
        img = synth.make_image(size[0], size[1], regions, 10.0, seed0 + b)
        labs.append(img.lab)
        # spread the contour so that dw/dC is not ~0 almost everywhere
        c = img.contour + 0.2 * np.random.default_rng(seed0 + b).random(img.contour.shape)
        cons.append(np.clip(c, 0, 1).astype(np.float32))
    return np.stack(labs), np.stack(cons)


def _endpoint_margin(theta):
    """Distance from a rounding boundary of the soft barycenter coordinates that a
    later iteration rounds to a path endpoint.  Coordinates exactly on a half are
    excluded: in FP64 that needs every other soft weight to underflow to 0
    (D gaps above 745 T), far beyond FP32's underflow, so the GPU lands on the
    same half exactly and rounds the same way."""
    xy = theta[1:-1, ..., 3:5]
    d = np.abs(xy - np.floor(xy) - 0.5)
    d = d[d > 0]
    return float(d.min()) if d.size else float("inf")


def _engine(W, H, k, B, T, iters, **kw):
    from paper_1903_07149_amd.soft import SoftScalp
    return SoftScalp(W, H, k, B, temperature=T, iterations=iters, **kw)


U = 2.0 ** -24


def assert_grads(orc, lab, con, k, gq, gth, iters, T, glab, gcon, cut=True, **kw):
    """Element-wise check of the GPU gradients against the oracle's (see the
    module docstring); gq is [B][9][H][W] as the GPU takes it."""
    glab_o, gcon_o, bd = orc.soft_backward(lab, con, k, gq.transpose(0, 2, 3, 1), gth,
                                           iterations=iters, T=T, d32=True, qcut=cut, bound=True,
                                           **kw)
    for got, ref, (E, Md), name in ((glab, glab_o, bd["lab"], "lab"),
                                    (gcon, gcon_o, bd["contour"], "contour")):
        tol = U * E + Md + 1e-37
        err = np.abs(got - ref)
        ratio = err / tol
        i = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"grad {name}: worst element {tuple(int(v) for v in i)}: got {got[i]:.6e}, "
              f"ref {ref[i]:.6e}, |diff| {err[i]:.3e} = {ratio[i]:.3e} of its bound "
              f"{tol[i]:.3e}; median bound / max|ref| {np.median(tol) / np.abs(ref).max():.2e}; "
              f"relative L2 {rel:.3e}")
        assert (err <= tol).all(), (name, i)
        assert rel <= 1e-3, name


CASES = [  # (W, H, k, B, T, iterations, seed)
    (96, 80, 30, 2, 0.5, 3, 600),
    (64, 64, 16, 2, 5.0, 4, 610),
    (70, 45, 12, 1, 50.0, 2, 620),
]


def _round_xy(theta, W, H):
    xy = theta[..., 3:5]
    e = np.floor(xy + np.float32(0.5)) if xy.dtype == np.float32 else np.floor(xy + 0.5)
    return np.stack([np.clip(e[..., 0], 0, W - 1), np.clip(e[..., 1], 0, H - 1)], axis=-1)


def compare_forward(c_t, q_t, th_o, q_o, W, H):
    """Per-iteration comparison.  Iteration t is compared while the path endpoints
    both sides derive from Theta_{t-1} agree; where they first differ, the differing
    coordinates must lie within 1e-2 of a rounding half in the FP64 oracle (both
    roundings are then valid), and later iterations are not compared.
    Returns the number of iterations compared."""
    q_ref = q_o.transpose(0, 1, 4, 2, 3)            # -> [T][B][9][H][W]
    T = q_t.shape[0]
    for t in range(T):
        eg = _round_xy(c_t[t], W, H)
        eo = _round_xy(th_o[t], W, H)
        if not (eg == eo).all():
            bad = eg != eo
            frac = th_o[t][..., 3:5] - np.floor(th_o[t][..., 3:5])
            print(f"iteration {t + 1}: {int(bad.sum())} endpoint coordinates round differently")
            assert (np.abs(frac - 0.5)[bad] < 1e-2).all()
            return t
        dq = np.abs(q_t[t] - q_ref[t]).max()
        dth = (np.abs(c_t[t + 1] - th_o[t + 1]) / (np.abs(th_o[t + 1]) + 1.0)).max()
        print(f"iteration {t + 1}: max |dQ| = {dq:.3e}, max rel dTheta = {dth:.3e}")
        assert dq <= 1e-6, t
        assert dth <= 1e-6, t
    return T


@pytest.mark.parametrize("T", [0.5, 0.05, 5.0])
def test_soft_pruning_changes_no_bit(T):
    """exact_pruning skips only slots whose softmax weight is provably 0: Q
    and the centres are bit-identical with and without it; the gradients
    agree to the rounding of the backward's float atomics."""
    W, H, k, B, iters = 160, 120, 40, 2, 3
    lab, con = _batch(B, (W, H), 8, 640)
    outs = []
    for prune in (1, 0):
        eng = _engine(W, H, k, B, T, iters, exact_pruning=prune)
        say("soft pruning", prune, T)
        L, C = dev(lab), dev(con)
        c_t, q_t, saved = eng.forward(L, C)
        gq = torch.from_numpy(np.random.default_rng(5).standard_normal(tuple(q_t[-1].shape)).astype(np.float32)).cuda()
        gth = torch.from_numpy(np.random.default_rng(6).standard_normal(tuple(c_t[-1].shape)).astype(np.float32)).cuda()
        glab, gcon = eng.backward(L, C, c_t, q_t, saved, gq, gth)
        outs.append([host(t) for t in (c_t, q_t, glab, gcon)])
    for a, b in zip(outs[0][:2], outs[1][:2]):
        assert np.array_equal(a, b)
    for a, b in zip(outs[0][2:], outs[1][2:]):
        assert np.allclose(a, b, rtol=1e-5, atol=1e-6 * max(1.0, float(np.abs(b).max())))


@pytest.mark.parametrize("W,H,k,B,T,iters,seed", CASES)
def test_soft_forward_matches_oracle(orc, W, H, k, B, T, iters, seed):
    lab, con = _batch(B, (W, H), 8, seed)
    th_o, q_o, z_o = orc.soft_forward(lab, con, k, iterations=iters, T=T, d32=True)
    eng = _engine(W, H, k, B, T, iters)
    say("soft forward", W, H, k, B, T, iters)
    c_t, q_t, saved = eng.forward(dev(lab), dev(con))
    c_t, q_t = host(c_t), host(q_t)
    assert compare_forward(c_t, q_t, th_o, q_o, W, H) == iters
    assert np.allclose(q_t.sum(axis=2), 1.0, atol=1e-5)


@pytest.mark.parametrize("wg", [256, 512, 1024])
def test_soft_forward_sliced_cells(orc, wg):
    """Cells of 32 x 40 = 1280 pixels exceed every workgroup size, so each is cut
    into 5, 3 or 2 work items of whole 64-pixel chunks."""
    W, H, k, B, T, iters, seed = 96, 80, 6, 2, 0.5, 2, 630
    lab, con = _batch(B, (W, H), 8, seed)
    th_o, q_o, z_o = orc.soft_forward(lab, con, k, iterations=iters, T=T, d32=True)
    eng = _engine(W, H, k, B, T, iters, wg_size=wg)
    assert (eng.grid.nx, eng.grid.ny) == (3, 2)
    say("soft forward sliced", wg)
    c_t, q_t, saved = eng.forward(dev(lab), dev(con))
    c_t, q_t = host(c_t), host(q_t)
    assert compare_forward(c_t, q_t, th_o, q_o, W, H) == iters


def test_soft_forward_wide_axis(orc):
    """A 70000-pixel-wide image: the per-pixel soft kernels find their cell with
    the 64-bit branch of the cell arithmetic."""
    W, H, k, B, T, iters, seed = 70000, 2, 40, 1, 5.0, 2, 640
    lab, con = _batch(B, (W, H), 40, seed)
    th_o, q_o, z_o = orc.soft_forward(lab, con, k, iterations=iters, T=T, d32=True)
    eng = _engine(W, H, k, B, T, iters)
    say("soft forward wide", W, H, k)
    c_t, q_t, saved = eng.forward(dev(lab), dev(con))
    c_t, q_t = host(c_t), host(q_t)
    assert compare_forward(c_t, q_t, th_o, q_o, W, H) == iters


@pytest.mark.parametrize("W,H,k,B,T,iters,seed", CASES)
def test_soft_backward_matches_oracle(orc, W, H, k, B, T, iters, seed):
    lab, con = _batch(B, (W, H), 8, seed)
    rng = np.random.default_rng(seed + 1)
    K = orc.grid(W, H, k).num_sp
    gq = rng.normal(0, 1, (B, 9, H, W)).astype(np.float32)
    gth = rng.normal(0, 1, (B, K, 5)).astype(np.float32)
    eng = _engine(W, H, k, B, T, iters)
    L, C = dev(lab), dev(con)
    say("soft backward", W, H, k, B, T, iters)
    c_t, q_t, saved = eng.forward(L, C)
    glab, gcon = (host(t) for t in eng.backward(L, C, c_t, q_t, saved, dev(gq), dev(gth)))
    assert_grads(orc, lab, con, k, gq, gth, iters, T, glab, gcon)


def test_soft_backward_near_the_cut(orc):
    """T = 2: a few per cent of the nonzero Q lie within a factor 16 of 2^-24.
    Element-wise against the oracle with the cut, and against the plain chain
    rule within the bound of what the cut changes."""
    W, H, k, B, T, iters, seed = 96, 80, 30, 1, 2.0, 3, 660
    lab, con = _batch(B, (W, H), 8, seed)
    rng = np.random.default_rng(seed + 1)
    K = orc.grid(W, H, k).num_sp
    gq = rng.normal(0, 1, (B, 9, H, W)).astype(np.float32)
    gth = rng.normal(0, 1, (B, K, 5)).astype(np.float32)
    _, q_o, _ = orc.soft_forward(lab, con, k, iterations=iters, T=T, d32=True)
    qv = q_o[q_o > 0]
    assert np.count_nonzero((qv > 2.0 ** -28) & (qv < 2.0 ** -20)) >= 0.01 * qv.size
    eng = _engine(W, H, k, B, T, iters)
    L, C = dev(lab), dev(con)
    say("soft backward near the cut", T)
    c_t, q_t, saved = eng.forward(L, C)
    glab, gcon = (host(t) for t in eng.backward(L, C, c_t, q_t, saved, dev(gq), dev(gth)))
    assert_grads(orc, lab, con, k, gq, gth, iters, T, glab, gcon, cut=True)
    assert_grads(orc, lab, con, k, gq, gth, iters, T, glab, gcon, cut=False)


def test_autograd_function_and_lds_fallback(orc):
    from paper_1903_07149_amd.soft import scalp_soft
    W, H, k, B, T, iters = 80, 64, 20, 2, 2.0, 3
    lab, con = _batch(B, (W, H), 6, 700)
    rng = np.random.default_rng(5)
    K = orc.grid(W, H, k).num_sp
    gq = rng.normal(0, 1, (B, 9, H, W)).astype(np.float32)
    gth = rng.normal(0, 1, (B, K, 5)).astype(np.float32)
    results = []
    # default; no LDS tables; partial; the largest budget (the backward's
    # tiles are capped below it)
    for lds in (0, 1, 300, 9728):
        eng = _engine(W, H, k, B, T, iters, lds_pixels=lds)
        L = dev(lab).requires_grad_(True)
        C = dev(con).requires_grad_(True)
        say("autograd", lds)
        q, th = scalp_soft(L, C, eng)
        loss = (q * dev(gq)).sum() + (th * dev(gth)).sum()
        loss.backward()
        results.append((host(L.grad), host(C.grad)))
    for glab, gcon in results:
        assert_grads(orc, lab, con, k, gq, gth, iters, T, glab, gcon)


def test_soft_large_cells_largest_budget(orc):
    """64x64-pixel cells with the largest LDS budget: the forward stages every
    candidate's table, while the backward stages the own cell's weight tile
    and scatters the other slots' paths (whose boxes no longer fit its capped
    budget) to global memory.  At T = 50 the softmax is far from one-hot, so
    both gradients are large."""
    W, H, k, B, T, iters = 128, 128, 4, 1, 50.0, 2
    lab, con = _batch(B, (W, H), 6, 720)
    rng = np.random.default_rng(6)
    K = orc.grid(W, H, k).num_sp
    assert K == 4
    gq = rng.normal(0, 1, (B, 9, H, W)).astype(np.float32)
    gth = rng.normal(0, 1, (B, K, 5)).astype(np.float32)
    th_o, q_o, _ = orc.soft_forward(lab, con, k, iterations=iters, T=T, d32=True)
    eng = _engine(W, H, k, B, T, iters, lds_pixels=9728)
    say("soft large cells, lds 9728")
    L, C = dev(lab), dev(con)
    c_t, q_t, saved = eng.forward(L, C)
    glab, gcon = (host(t) for t in eng.backward(L, C, c_t, q_t, saved, dev(gq), dev(gth)))
    assert compare_forward(host(c_t), host(q_t), th_o, q_o, W, H) == iters
    assert_grads(orc, lab, con, k, gq, gth, iters, T, glab, gcon)


def test_soft_low_temperature_is_hard(orc):
    """Integer Lab on 4x4-pixel cells: T -> 0 gives one-hot Q at the hard assignment."""
    from paper_1903_07149_amd.scalp import Scalp
    W = H = 16
    rng = np.random.default_rng(4)
    lab = rng.integers(0, 60, (H, W, 3)).astype(np.float32)
    con = (rng.integers(0, 5, (H, W)) / 4.0).astype(np.float32)
    eng = _engine(W, H, 16, 1, 1e-3, 1)
    say("soft T->0")
    c_t, q_t, _ = eng.forward(dev(lab[None]), dev(con[None]))
    s = Scalp(W, H, 16)
    c0, e0, _ = s.init_grid(dev(lab), dev(con))
    assert (host(c_t)[0, 0] == host(c0)).all()
    hard = host(s.assign(dev(lab), dev(con), c0, e0))
    g = orc.grid(W, H, 16)
    yy, xx = np.mgrid[0:H, 0:W]
    j = host(q_t)[0, 0].argmax(axis=0)
    soft_lbl = (yy * g.ny // H + j // 3 - 1) * g.nx + (xx * g.nx // W + j % 3 - 1)
    assert (soft_lbl == hard).all()


def test_soft_full_size_workload(orc):
    """The benchmark's soft workload (16 x 512x512, k = 400, T = 0.5, 5 iterations),
    forward and backward in one launch configuration: invariants on the whole batch,
    and image 3 of the batch against the oracle."""
    orc.set_threads(min(16, os.cpu_count() or 1))
    wls = synth.soft_workloads()
    imgs = [synth.workload_image(w) for w in wls]
    lab = np.stack([i.lab for i in imgs])
    con = np.stack([i.contour for i in imgs])
    L, C = dev(lab), dev(con)
    rng = np.random.default_rng(9)
    K = orc.grid(512, 512, 400).num_sp
    gq = rng.normal(0, 1, (16, 9, 512, 512)).astype(np.float32)
    gth = rng.normal(0, 1, (16, K, 5)).astype(np.float32)
    eng = _engine(512, 512, 400, 16, 0.5, 5)
    say("soft full size, 5 iterations")
    c_t, q_t, saved = eng.forward(L, C)
    glab, gcon = (host(t) for t in eng.backward(L, C, c_t, q_t, saved, dev(gq), dev(gth)))
    c_t, q_t = host(c_t), host(q_t)
    assert np.allclose(q_t.sum(axis=2), 1.0, atol=1e-5) and (q_t >= 0).all()
    assert np.isfinite(glab).all() and np.isfinite(gcon).all()
    assert (c_t[..., 3] >= 0).all() and (c_t[..., 3] <= 511).all()
    assert (c_t[..., 4] >= 0).all() and (c_t[..., 4] <= 511).all()
    i = 3
    th_o, q_o, _ = orc.soft_forward(lab[i:i + 1], con[i:i + 1], 400, iterations=5, T=0.5, d32=True)
    assert compare_forward(c_t[:, i:i + 1], q_t[:, i:i + 1], th_o, q_o, 512, 512) == 5
    assert_grads(orc, lab[i:i + 1], con[i:i + 1], 400, gq[i:i + 1], gth[i:i + 1], 5, 0.5,
                 glab[i:i + 1], gcon[i:i + 1])
