"""Window form of the assignment (the candidate rule of Algorithm 1) on the GPU against
the oracle: one pass bit-exact (labels, with uncovered pixels keeping theirs),
whole runs bit-exact against the fixed-point-mean oracle and >= 99.9 % label
agreement against the FP64-mean oracle.  Also reports how far the window form
and the 3x3 grid form end up from each other."""
import os

import numpy as np
import pytest

from paper_1903_07149_amd import synth
from paper_1903_07149_amd._lib import ASSIGN_WINDOW
from gpu_util import dev, host, needs_gpu, perturbed_state, say, torch

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.fixture(scope="module", autouse=True)
def _threads(orc):
    orc.set_threads(min(16, os.cpu_count() or 1))


def _scalp(W, H, k, **kw):
    from paper_1903_07149_amd.scalp import Scalp
    return Scalp(W, H, k, assign_mode=ASSIGN_WINDOW, **kw)


CASES = [(97, 61, 30), (481, 321, 250), (37, 5, 7), (1, 1, 1), (64, 64, 4096), (300, 200, 2)]
TUNINGS = [dict(), dict(lds_pixels=1), dict(wg_size=256, lds_pixels=900)]


@pytest.mark.parametrize("tune", range(len(TUNINGS)))
@pytest.mark.parametrize("W,H,k", CASES)
def test_window_assign_bit_exact(orc, W, H, k, tune):
    img = synth.make_image(W, H, max(2, W * H // 4000), 10.0, 13)
    g = orc.grid(W, H, k)
    c, e = perturbed_state(orc, g, img.lab, seed=W + 3 * H, jitter=0.3 * g.r + 1)
    prev = np.random.default_rng(1).integers(0, g.num_sp, (H, W)).astype(np.int32)
    s = _scalp(W, H, k, **TUNINGS[tune])
    say("window assign", W, H, k, TUNINGS[tune])
    lbl = host(s.assign(dev(img.lab), dev(img.contour), dev(c), dev(e), labels=dev(prev)))
    ol, _ = orc.assign_window(g, img.lab, orc.wmap(img.contour), c, e, prev)
    assert (lbl == ol).all(), f"{int((lbl != ol).sum())} labels differ"


def _compare(orc, img, k, iters):
    H, W = img.contour.shape
    s = _scalp(W, H, k)
    say("window run", W, H, k, iters)
    r = s.run(dev(img.lab), dev(img.contour), iterations=iters)
    lbl, c, e = host(r.labels), host(r.centers), host(r.endpoints)
    fixed = orc.run_window(img.lab, img.contour, k, iterations=iters, mode=orc.MEAN_FIXED)
    assert (lbl == fixed.labels).all(), f"{int((lbl != fixed.labels).sum())} labels differ"
    assert (c == fixed.centres).all() and (e == fixed.endpoints).all()
    plain = orc.run_window(img.lab, img.contour, k, iterations=iters, mode=orc.MEAN_PLAIN)
    assert (lbl == plain.labels).mean() >= 0.999
    grid3 = orc.run(img.lab, img.contour, k, iterations=iters, mode=orc.MEAN_FIXED)
    agree = float((lbl == grid3.labels).mean())
    print(f"{W}x{H} k={k}: window form vs 3x3 form label agreement {agree:.4f}")
    return agree


@pytest.mark.parametrize("W,H,k", [(97, 61, 30), (160, 120, 48)])
def test_window_run_small(orc, W, H, k):
    _compare(orc, synth.make_image(W, H, 6, 10.0, 21), k, 10)


def test_window_run_bsd_shape(orc):
    _compare(orc, synth.workload_image(synth.BSD_SHAPE), 250, 10)


def test_window_run_hd(orc):
    _compare(orc, synth.workload_image(synth.HD), synth.HD.k, 10)


def test_window_graph_replays(orc):
    img = synth.make_image(200, 150, 8, 10.0, 3)
    s = _scalp(200, 150, 60)
    lab, con = dev(img.lab), dev(img.contour)
    say("window graph")
    ref = s.run(lab, con)
    refs = [host(t) for t in (ref.labels, ref.centers, ref.endpoints)]
    c, e, l = s.init_grid(lab, con)
    n = torch.empty_like(ref.counts)
    gr = s.graph(c, e, l, n)
    for rep in range(3):
        s.init_grid(lab, con, out=(c, e, l))
        torch.cuda.synchronize()
        gr.launch()
        for a, b in zip((host(l), host(c), host(e)), refs):
            assert (a == b).all(), rep
    gr.close()


def test_window_mode_rejected_where_unsupported():
    from paper_1903_07149_amd import _lib as L
    from paper_1903_07149_amd.scalp import ScalpBatch
    from paper_1903_07149_amd.soft import SoftScalp
    b = ScalpBatch([(40, 30, 12)], assign_mode=ASSIGN_WINDOW)
    lab = torch.zeros((1200, 3), device="cuda")
    con = torch.zeros((1200,), device="cuda")
    with pytest.raises(L.ScalpError) as ei:
        b.run(lab, con)
    assert ei.value.code == L.SCALP_ERR_UNSUPPORTED
    eng = SoftScalp(32, 32, 16, 1, assign_mode=ASSIGN_WINDOW)
    with pytest.raises(L.ScalpError):
        eng.forward(torch.zeros((1, 32, 32, 3), device="cuda"), torch.zeros((1, 32, 32), device="cuda"))
