"""Batched hard SCALP (one persistent launch per iteration over a ragged batch
of images) gives, per image, exactly the single-image results, eagerly and
as a replayed hipGraph."""
import os

import numpy as np
import pytest

from paper_1903_07149_amd import synth
from gpu_util import dev, host, needs_gpu, say, torch

pytestmark = [pytest.mark.gpu, needs_gpu]


def _batch(n, seed0, lo, hi, per_px):
    return synth.batch_workloads(n=n, seed0=seed0, lo=lo, hi=hi, per_px=per_px)


@pytest.mark.parametrize("tune", [dict(), dict(wg_size=256), dict(wg_size=512),
                                  dict(lds_pixels=700), dict(exact_pruning=0),
                                  dict(persistent_blocks=1), dict(wg_size=256, persistent_blocks=3),
                                  dict(table_mode=1), dict(table_mode=1, lds_pixels=700, wg_size=512)])
def test_batched_equals_single_and_oracle(orc, tune):
    from paper_1903_07149_amd.scalp import Scalp, ScalpBatch
    orc.set_threads(min(16, os.cpu_count() or 1))
    wls = _batch(7, 900, 30, 260, 300)
    wls.append(synth.Workload("one_px", 1, 1, 1, 10.0, 1, 1, 10))
    wls.append(synth.Workload("single_sp", 90, 40, 3, 10.0, 2, 1, 10))
    # cells of 150x200 pixels: each is split into several work items
    wls.append(synth.Workload("big_cells", 300, 200, 5, 10.0, 3, 2, 10))
    imgs = [synth.workload_image(w) for w in wls]
    b = ScalpBatch([(w.width, w.height, w.k) for w in wls], iterations=6, **tune)
    lab = dev(np.concatenate([i.lab.reshape(-1, 3) for i in imgs]))
    con = dev(np.concatenate([i.contour.reshape(-1) for i in imgs]))
    say("batched", tune)
    c, e, l, n = (host(t) for t in b.run(lab, con))
    for (p0, p1, H, W), (s0, s1), w, img in zip(b.pixel_slices(), b.sp_slices(), wls, imgs):
        s = Scalp(W, H, w.k, iterations=6, **tune)
        r = s.run(dev(img.lab), dev(img.contour))
        assert (l[p0:p1].reshape(H, W) == host(r.labels)).all(), w.name
        assert (c[s0:s1] == host(r.centers)).all() and (e[s0:s1] == host(r.endpoints)).all()
        assert (n[s0:s1] == host(r.counts)).all()
        ref = orc.run(img.lab, img.contour, w.k, iterations=6, mode=orc.MEAN_FIXED)
        assert (l[p0:p1].reshape(H, W) == ref.labels).all(), w.name


def test_batched_graph_replays():
    from paper_1903_07149_amd.scalp import ScalpBatch
    wls = _batch(5, 950, 40, 300, 500)
    imgs = [synth.workload_image(w) for w in wls]
    b = ScalpBatch([(w.width, w.height, w.k) for w in wls], iterations=5)
    lab = dev(np.concatenate([i.lab.reshape(-1, 3) for i in imgs]))
    con = dev(np.concatenate([i.contour.reshape(-1) for i in imgs]))
    say("batched graph")
    ref = [host(t) for t in b.run(lab, con)]
    st = b.new_state()
    gr = b.graph(lab, con, *st)
    for rep in range(3):
        for t in st:
            t.fill_(-7)                           # eager work between replays
        torch.cuda.synchronize()
        gr.launch()
        got = [host(t) for t in st]
        for a, r in zip(got, ref):
            assert (a == r).all(), rep
    gr.close()


@pytest.mark.timeout(400)   # generating the 64 images takes most of it
def test_batched_full_size_workload(orc):
    """The benchmark's batch (64 ragged images, 92 Mpx, k = HW/1000, 10 iterations)
    in the launch shape the benchmark uses (the autotuner's choice for this
    batch): every image equals the single-image path bit for bit, and three
    sampled images (the smallest, a middle one and the largest) equal the
    oracle."""
    from paper_1903_07149_amd import autotune
    from paper_1903_07149_amd.scalp import Scalp, ScalpBatch
    orc.set_threads(min(16, os.cpu_count() or 1))
    wls = synth.batch_workloads()
    assert len(wls) == 64
    imgs = [synth.workload_image(w) for w in wls]
    shapes = [(w.width, w.height, w.k) for w in wls]
    lab = dev(np.concatenate([i.lab.reshape(-1, 3) for i in imgs]))
    con = dev(np.concatenate([i.contour.reshape(-1) for i in imgs]))
    say("batched full size: tuning")
    tuned = autotune.tune_batch(shapes, lab, con, use_cache=False)
    assert tuned in autotune.BATCH_CANDIDATES
    b = ScalpBatch(shapes, iterations=10, **tuned)
    say("batched full size", tuned)
    c, e, l, n = (host(t) for t in b.run(lab, con))
    del lab, con
    sizes = [w.width * w.height for w in wls]
    order = np.argsort(sizes)
    sampled = {int(order[0]), int(order[len(order) // 2]), int(order[-1])}
    slices = list(zip(b.pixel_slices(), b.sp_slices()))
    for i, (w, img) in enumerate(zip(wls, imgs)):
        (p0, p1, H, W), (s0, s1) = slices[i]
        s = Scalp(W, H, w.k, iterations=10)
        r = s.run(dev(img.lab), dev(img.contour))
        assert (l[p0:p1].reshape(H, W) == host(r.labels)).all(), w.name
        assert (c[s0:s1] == host(r.centers)).all() and (e[s0:s1] == host(r.endpoints)).all()
        assert (n[s0:s1] == host(r.counts)).all()
        if i in sampled:
            say("oracle", w.name)
            ref = orc.run(img.lab, img.contour, w.k, iterations=10, mode=orc.MEAN_FIXED)
            assert (l[p0:p1].reshape(H, W) == ref.labels).all(), w.name
            assert (c[s0:s1] == ref.centres).all() and (e[s0:s1] == ref.endpoints).all()


@pytest.mark.parametrize("W,H,k", [(481, 321, 250), (129, 77, 1), (1920, 1080, 2000)])
def test_batched_single_image_equals_single_path(W, H, k):
    """A batch of one image: every XCD's run of work items is a share of the
    same image, and the results equal the single-image path's."""
    from paper_1903_07149_amd.scalp import Scalp, ScalpBatch
    wl = synth.Workload(f"one_{W}x{H}", W, H, 40, 10.0, 7, k, 5)
    img = synth.workload_image(wl)
    say("batch of one", W, H, k)
    b = ScalpBatch([(W, H, k)], iterations=5)
    c, e, l, n = (host(t) for t in b.run(dev(img.lab.reshape(-1, 3)), dev(img.contour.reshape(-1))))
    r = Scalp(W, H, k, iterations=5).run(dev(img.lab), dev(img.contour))
    assert (l.reshape(H, W) == host(r.labels)).all()
    assert (c == host(r.centers)).all() and (e == host(r.endpoints)).all()
    assert (n == host(r.counts)).all()
