"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars:
  * packed w map, grid initialisation, one assignment pass from identical
    centres, and the update from identical labels: bit-exact;
  * whole runs: bit-exact against the oracle's fixed-point-mean mode (the
    same rounding of the mean as the GPU's order-free integer sums), and at
    least 99.9 % label agreement with barycenters within 1e-5 relative
    against the oracle's plain FP64 mean.
"""
import os

import numpy as np
import pytest

from paper_1903_07149_amd import synth
from gpu_util import dev, host, needs_gpu, perturbed_state, say, torch

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.fixture(scope="module", autouse=True)
def _threads(orc):
    orc.set_threads(min(16, os.cpu_count() or 1))


def _image(W, H, seed, regions=None):
    if regions is None:
        regions = max(2, (W * H) // 4000)
    return synth.make_image(W, H, regions, 10.0, seed)


# (W, H, k): several tiles and ragged cells, thin and degenerate shapes,
# one superpixel per pixel, and cells too large for the LDS tables.
SMALL = [(97, 61, 30), (256, 200, 100), (481, 321, 250), (37, 5, 7), (1, 1, 1), (1, 50, 5),
         (50, 1, 5), (64, 64, 4096), (300, 200, 2), (129, 77, 1)]
# tuning variants: default (1024 threads, 4800-unit LDS tables); tables too small for
# most endpoints; budget below one cell (every path from global memory);
# 256- and 512-thread workgroups; tables voted down to the walking waves' box
# (alone, with a small budget, and with every candidate walked)
TUNINGS = [dict(), dict(lds_pixels=900), dict(lds_pixels=1), dict(wg_size=256),
           dict(wg_size=512, lds_pixels=3200), dict(table_mode=1),
           dict(table_mode=1, wg_size=256, lds_pixels=900),
           dict(table_mode=1, exact_pruning=0, wg_size=512)]


def _scalp(W, H, k, **kw):
    from paper_1903_07149_amd.scalp import Scalp
    return Scalp(W, H, k, **kw)


@pytest.mark.parametrize("W,H,k", SMALL[:4])
def test_prepare_packs_w_bit_exact(orc, W, H, k):
    img = _image(W, H, 1)
    con = img.contour.copy()
    con.ravel()[::7] = np.random.default_rng(0).random(con.size)[::7]   # many distinct values
    s = _scalp(W, H, k)
    say("prepare", W, H, k)
    s.prepare(dev(img.lab), dev(con))
    packed = host(s.workspace[: 16 * W * H].view(torch.float32)).reshape(H, W, 4)
    assert (packed[..., :3] == img.lab).all()
    w = orc.wmap(con)
    mism = int((packed[..., 3] != w).sum())
    assert mism == 0, f"{mism} w values differ"


@pytest.mark.parametrize("W,H,k", SMALL)
def test_init_grid_bit_exact(orc, W, H, k):
    img = _image(W, H, 2)
    s = _scalp(W, H, k)
    g = orc.grid(W, H, k)
    say("init_grid", W, H, k)
    c, e, l = s.init_grid(dev(img.lab), dev(img.contour))
    oc, oe, ol = orc.init_grid(g, img.lab, mode=orc.MEAN_FIXED)
    assert (host(l) == ol).all()
    assert (host(c) == oc).all()
    assert (host(e) == oe).all()


@pytest.mark.parametrize("tune", range(len(TUNINGS)))
@pytest.mark.parametrize("W,H,k", SMALL)
def test_assign_bit_exact(orc, W, H, k, tune):
    img = _image(W, H, 3)
    g = orc.grid(W, H, k)
    c, e = perturbed_state(orc, g, img.lab, seed=W * 7 + H, jitter=0.3 * g.r + 1)
    s = _scalp(W, H, k, **TUNINGS[tune])
    say("assign", W, H, k, TUNINGS[tune])
    lbl = host(s.assign(dev(img.lab), dev(img.contour), dev(c), dev(e)))
    ol, _, _ = orc.assign(g, img.lab, orc.wmap(img.contour), c, e)
    assert (lbl == ol).all(), f"{int((lbl != ol).sum())} labels differ"


@pytest.mark.parametrize("W,H,k,tune", [(2100, 1000, 1, {}), (3000, 3, 2, {"lds_pixels": 9728}),
                                         (2, 2600, 1, {})])
def test_assign_long_paths(orc, W, H, k, tune):
    """One 2100x1000 cell: paths of up to ~1050 samples, walked from global
    memory, whose averages over more than 1024 samples take the IEEE
    divisions; thin images: many short cells, tables of extreme aspect."""
    img = _image(W, H, 8, regions=6)
    g = orc.grid(W, H, k)
    c, e = perturbed_state(orc, g, img.lab, seed=W + H, jitter=2.0)
    s = _scalp(W, H, k, **tune)
    say("assign long paths", W, H, k, tune)
    lbl = host(s.assign(dev(img.lab), dev(img.contour), dev(c), dev(e)))
    ol, _, _ = orc.assign(g, img.lab, orc.wmap(img.contour), c, e)
    assert (lbl == ol).all(), f"{int((lbl != ol).sum())} labels differ"


@pytest.mark.parametrize("W,H,k,tune", [(481, 321, 30, {"lds_pixels": 1100}),
                                         (600, 600, 4, {}),
                                         (600, 600, 4, {"wg_size": 256, "lds_pixels": 4500}),
                                         (700, 500, 12, {"lds_pixels": 9728}),
                                         (97, 900, 3, {"wg_size": 512, "lds_pixels": 1000}),
                                         (481, 321, 30, {"lds_pixels": 1100, "table_mode": 1}),
                                         (600, 600, 4, {"table_mode": 1}),
                                         (700, 500, 12, {"lds_pixels": 9728, "table_mode": 1}),
                                         (97, 900, 3, {"wg_size": 256, "lds_pixels": 1000,
                                                       "table_mode": 1})])
def test_assign_tables_beyond_budget(orc, W, H, k, tune):
    """Cells whose table rectangles exceed the LDS budget by a few to tens of
    times (their paths read global memory) beside candidates whose tables
    fit, with endpoints jittered above, below and inside the cells."""
    img = _image(W, H, 11, regions=12)
    g = orc.grid(W, H, k)
    c, e = perturbed_state(orc, g, img.lab, seed=W * 3 + k, jitter=0.4 * g.r + 1)
    s = _scalp(W, H, k, **tune)
    say("assign tables beyond budget", W, H, k, tune)
    lbl = host(s.assign(dev(img.lab), dev(img.contour), dev(c), dev(e)))
    ol, _, _ = orc.assign(g, img.lab, orc.wmap(img.contour), c, e)
    assert (lbl == ol).all(), f"{int((lbl != ol).sum())} labels differ"


def test_assign_paths_beyond_carry_range(orc):
    """Caller-supplied endpoints of the last three superpixels of a 60000-pixel
    row at its left end: the paths to them from the right end have more than
    46340 steps (beyond the range of the carry-counting stepper) and take the
    exact remainder stepping of the global-memory walk."""
    W, H, k = 60000, 1, 100
    img = _image(W, H, 21, regions=30)
    g = orc.grid(W, H, k)
    c, e = perturbed_state(orc, g, img.lab, seed=5, jitter=2.0)
    e = e.copy()
    e[-3:] = 0
    s = _scalp(W, H, k)
    say("assign paths beyond 46340 steps")
    lbl = host(s.assign(dev(img.lab), dev(img.contour), dev(c), dev(e)))
    ol, _, _ = orc.assign(g, img.lab, orc.wmap(img.contour), c, e)
    assert (lbl == ol).all(), f"{int((lbl != ol).sum())} labels differ"


@pytest.mark.parametrize("scale", [1e-21, 1e-17])
def test_assign_tiny_colour_sums(orc, scale):
    """Lab values so small that the path colour sums fall below 2^-100 (down
    to the subnormal range): those averages take the IEEE division."""
    W, H, k = 97, 61, 30
    img = _image(W, H, 9)
    lab = (img.lab * np.float32(scale)).astype(np.float32)
    g = orc.grid(W, H, k)
    c, e = perturbed_state(orc, g, lab, seed=3, jitter=3.0, colour=10.0 * scale)
    s = _scalp(W, H, k)
    say("assign tiny", scale)
    lbl = host(s.assign(dev(lab), dev(img.contour), dev(c), dev(e)))
    ol, _, _ = orc.assign(g, lab, orc.wmap(img.contour), c, e)
    assert (lbl == ol).all(), f"{int((lbl != ol).sum())} labels differ"


@pytest.mark.parametrize("lam,gamma", [(1.0, 0.0), (0.0, 0.0), (0.3, 7.0)])
def test_assign_parameters(orc, lam, gamma):
    W, H, k = 200, 150, 60
    img = _image(W, H, 4)
    g = orc.grid(W, H, k)
    c, e = perturbed_state(orc, g, img.lab, seed=5, jitter=4)
    s = _scalp(W, H, k, lam=lam, gamma=gamma, m=7.0)
    say("assign params", lam, gamma)
    lbl = host(s.assign(dev(img.lab), dev(img.contour), dev(c), dev(e)))
    ol, _, _ = orc.assign(g, img.lab, orc.wmap(img.contour), c, e, lam=lam, gamma=gamma,
                          spw=orc.spatial_weight(g, 7.0))
    assert (lbl == ol).all()


def test_assign_non_finite_texels(orc):
    """A few NaN texels: a pixel whose own colour is NaN has no finite D and
    keeps its own cell; a path through a NaN texel gives a NaN D that never
    wins; the bound that prunes is NaN exactly when the pixel's own colour is
    (same labels as the oracle, pruning or not)."""
    W, H, k = 97, 61, 30
    img = _image(W, H, 12)
    g = orc.grid(W, H, k)
    c, e = perturbed_state(orc, g, img.lab, seed=8, jitter=3.0)
    lab = img.lab.copy()
    rng = np.random.default_rng(9)
    for _ in range(6):
        lab[rng.integers(0, H), rng.integers(0, W), rng.integers(0, 3)] = np.nan
    ol, _, _ = orc.assign(g, lab, orc.wmap(img.contour), c, e)
    for prune in (1, 0):
        s = _scalp(W, H, k, exact_pruning=prune)
        say("assign non-finite", prune)
        lbl = host(s.assign(dev(lab), dev(img.contour), dev(c), dev(e)))
        assert (lbl == ol).all(), f"{int((lbl != ol).sum())} labels differ"


@pytest.mark.parametrize("lam,gamma,m", [(0.5, 0.0, 10.0), (1.0, 0.0, 0.0), (0.5, 5.0, 0.0),
                                         (0.0, 3.0, 10.0)])
def test_assign_exact_ties(orc, lam, gamma, m):
    """Two flat colours and centres at the cell middles, so that many pixels
    tie exactly between candidates (equal colour distance and mirrored
    spatial distance) and the colour-plus-spatial lower bound often equals D:
    the first strict minimum in ascending k must come out whatever order the
    kernel visits the candidates in and whichever it skips."""
    W, H, k = 96, 64, 24                        # 6 x 4 cells of 16 x 16
    g = orc.grid(W, H, k)
    rng = np.random.default_rng(17)
    pick = np.kron(rng.integers(0, 2, (H // 8, W // 8)), np.ones((8, 8), np.int64))
    colours = np.array([[40.0, 10.0, -5.0], [60.0, -20.0, 15.0]], np.float32)
    lab = np.ascontiguousarray(colours[pick], dtype=np.float32)
    contour = np.zeros((H, W), np.float32)
    contour[:, 40:42] = 0.5
    c = np.zeros((g.num_sp, 5), np.float32)
    e = np.zeros((g.num_sp, 2), np.int32)
    for kk in range(g.num_sp):
        i, j = divmod(kk, g.nx)
        c[kk, :3] = colours[(i + j) % 2]
        c[kk, 3] = 16 * j + 7.5
        c[kk, 4] = 16 * i + 7.5
        e[kk] = (16 * j + 8, 16 * i + 8)
    s = _scalp(W, H, k, lam=lam, gamma=gamma, m=m)
    say("assign exact ties", lam, gamma, m)
    lbl = host(s.assign(dev(lab), dev(contour), dev(c), dev(e)))
    ol, _, _ = orc.assign(g, lab, orc.wmap(contour), c, e, lam=lam, gamma=gamma,
                          spw=orc.spatial_weight(g, m))
    assert (lbl == ol).all(), f"{int((lbl != ol).sum())} labels differ"


@pytest.mark.parametrize("W,H,k", [(97, 61, 30), (481, 321, 250), (64, 64, 4096), (300, 200, 2)])
def test_update_bit_exact(orc, W, H, k):
    img = _image(W, H, 5)
    g = orc.grid(W, H, k)
    c, e = perturbed_state(orc, g, img.lab, seed=11, jitter=0.4 * g.r + 1)
    labels, _, _ = orc.assign(g, img.lab, orc.wmap(img.contour), c, e)
    s = _scalp(W, H, k)
    say("update", W, H, k)
    nc, ne, cnt = (host(t) for t in s.update(dev(img.lab), dev(labels), dev(c), dev(e)))
    oc, ocnt = orc.update(g, img.lab, labels, c, mode=orc.MEAN_FIXED)
    oe, _ = orc.project(g, labels, oc, ocnt, e)
    assert (cnt == ocnt).all()
    assert (nc == oc).all()
    assert (ne == oe).all()
    pc, _ = orc.update(g, img.lab, labels, c, mode=orc.MEAN_PLAIN)
    nz = ocnt > 0
    assert np.allclose(nc[nz], pc[nz], rtol=1e-5, atol=1e-5)


def test_update_arbitrary_labels(orc):
    """Labels that are not grid neighbours (global-atomic path, full-image projection scan)."""
    W, H, k = 120, 90, 24
    img = _image(W, H, 6)
    g = orc.grid(W, H, k)
    rng = np.random.default_rng(3)
    labels = rng.integers(0, g.num_sp, (H, W)).astype(np.int32)
    labels[labels == 3] = 4
    labels[:5, :5] = -1                             # ignored
    c, e, _ = orc.init_grid(g, img.lab, mode=orc.MEAN_FIXED)
    s = _scalp(W, H, k)
    say("update arbitrary labels")
    nc, ne, cnt = (host(t) for t in s.update(dev(img.lab), dev(labels), dev(c), dev(e)))
    oc, ocnt = orc.update(g, img.lab, labels, c, mode=orc.MEAN_FIXED)
    oe, moved = orc.project(g, labels, oc, ocnt, e)
    assert moved > 0
    assert (cnt == ocnt).all() and (nc == oc).all() and (ne == oe).all()


def test_update_many_labels_per_cell(orc):
    """Random labels over 64 superpixels on a 64x64 image: each 8x8 cell holds
    more distinct labels than the update's per-cell LDS table (32 slots), so
    the overflow goes to the global sums; results stay exact."""
    W, H, k = 64, 64, 64
    img = _image(W, H, 10)
    g = orc.grid(W, H, k)
    rng = np.random.default_rng(11)
    labels = rng.integers(0, g.num_sp, (H, W)).astype(np.int32)
    c, e, _ = orc.init_grid(g, img.lab, mode=orc.MEAN_FIXED)
    s = _scalp(W, H, k)
    say("update many labels per cell")
    nc, ne, cnt = (host(t) for t in s.update(dev(img.lab), dev(labels), dev(c), dev(e)))
    oc, ocnt = orc.update(g, img.lab, labels, c, mode=orc.MEAN_FIXED)
    oe, _ = orc.project(g, labels, oc, ocnt, e)
    assert (cnt == ocnt).all() and (nc == oc).all() and (ne == oe).all()


def _compare_runs(orc, img, k, iters, **kw):
    H, W = img.contour.shape
    s = _scalp(W, H, k, **kw)
    say("run", W, H, k, iters, kw)
    r = s.run(dev(img.lab), dev(img.contour), iterations=iters)
    lbl, c, e, n = host(r.labels), host(r.centers), host(r.endpoints), host(r.counts)
    fixed = orc.run(img.lab, img.contour, k, iterations=iters, mode=orc.MEAN_FIXED)
    assert (lbl == fixed.labels).all(), f"{int((lbl != fixed.labels).sum())} labels differ"
    assert (c == fixed.centres).all() and (e == fixed.endpoints).all()
    assert (n == fixed.counts).all()
    plain = orc.run(img.lab, img.contour, k, iterations=iters, mode=orc.MEAN_PLAIN)
    agree = float((lbl == plain.labels).mean())
    assert agree >= 0.999, agree
    return agree


@pytest.mark.parametrize("W,H,k", [(481, 321, 250), (97, 61, 30), (129, 77, 1), (64, 64, 4096)])
def test_run_bit_exact_small(orc, W, H, k):
    _compare_runs(orc, _image(W, H, 7), k, 10)


@pytest.mark.parametrize("W,H,k", [(70000, 3, 60), (3, 66000, 40)])
def test_run_bit_exact_wide_axis(orc, W, H, k):
    """An axis of 2^16 pixels or more takes the 64-bit branch of the cell
    arithmetic (below that, every product fits 32 bits)."""
    _compare_runs(orc, _image(W, H, 17, regions=40), k, 4)


def test_run_bsd_shape_workload(orc):
    _compare_runs(orc, synth.workload_image(synth.BSD_SHAPE), 250, 10)


def test_run_hd_workload(orc):
    """The benchmark's workload (1920x1080, k = 2000, 10 iterations) in its launch config."""
    _compare_runs(orc, synth.workload_image(synth.HD), synth.HD.k, synth.HD.iterations)


def test_run_bsd_shape_without_pruning(orc):
    """Every candidate walked (exact_pruning = 0): the same labels, centres and
    endpoints as the oracle, like the pruned default."""
    _compare_runs(orc, synth.workload_image(synth.BSD_SHAPE), 250, 10, exact_pruning=0)


def test_run_uhd_workload(orc):
    _compare_runs(orc, synth.workload_image(synth.UHD), synth.UHD.k, synth.UHD.iterations)


def test_graph_replays_match_eager(orc):
    img = synth.workload_image(synth.BSD_SHAPE)
    H, W = img.contour.shape
    s = _scalp(W, H, 250)
    lab, con = dev(img.lab), dev(img.contour)
    say("graph replay")
    ref = s.run(lab, con)
    refs = [host(t) for t in (ref.labels, ref.centers, ref.endpoints, ref.counts)]
    c, e, l = s.init_grid(lab, con)
    n = torch.empty_like(ref.counts)
    gr = s.graph(c, e, l, n)
    for rep in range(3):
        c0, e0, _ = s.init_grid(lab, con)          # eager work between replays
        c.copy_(c0)
        e.copy_(e0)
        torch.cuda.synchronize()
        gr.launch()
        got = [host(t) for t in (l, c, e, n)]
        for a, b in zip(got, refs):
            assert (a == b).all(), rep
    gr.close()


def test_run_repeatable_and_resumable(orc):
    img = _image(160, 120, 9)
    s = _scalp(160, 120, 48)
    lab, con = dev(img.lab), dev(img.contour)
    say("repeat/resume")
    a = s.run(lab, con, iterations=6)
    b = s.run(lab, con, iterations=6)
    for x, y in zip((a.labels, a.centers, a.endpoints), (b.labels, b.centers, b.endpoints)):
        assert (host(x) == host(y)).all()
    # 3 iterations, then 3 more from the saved state through a graph of the loop
    h = s.run(lab, con, iterations=3)
    c, e = h.centers.clone(), h.endpoints.clone()
    l, n = torch.empty_like(h.labels), torch.empty_like(h.counts)
    g3 = s.graph(c, e, l, n, iterations=3)
    g3.launch()
    assert (host(l) == host(a.labels)).all() and (host(c) == host(a.centers)).all()
    g3.close()
