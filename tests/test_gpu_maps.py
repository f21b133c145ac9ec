"""Per-pixel maps on the GPU against the oracle: the boundary-frequency map,
the contour prior computed from the image (standalone and fused into the
packing step, single and batched), and the 12-scale decomposition of one
image run as one batch."""
import os

import numpy as np
import pytest

from oracle import maps as OM
from paper_1903_07149_amd import synth
from paper_1903_07149_amd._lib import CONTOUR_GRADIENT
from gpu_util import dev, host, needs_gpu, say, torch

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.fixture(scope="module", autouse=True)
def _threads(orc):
    orc.set_threads(min(16, os.cpu_count() or 1))


@pytest.mark.parametrize("n,H,W,seed", [(1, 1, 1, 1), (3, 1, 70, 2), (2, 65, 1, 3), (12, 37, 53, 4),
                                        (5, 321, 481, 5)])
def test_boundary_map_bit_exact(n, H, W, seed):
    from paper_1903_07149_amd.maps import boundary_map
    rng = np.random.default_rng(seed)
    blk = np.kron(rng.integers(0, 6, (n, H // 3 + 1, W // 3 + 1)), np.ones((1, 3, 3)))
    L = blk[:, :H, :W].astype(np.int32)
    say("boundary map", n, H, W)
    got = host(boundary_map(dev(L)))
    assert (got == OM.boundary_frequency(L)).all()


@pytest.mark.parametrize("H,W,seed", [(1, 1, 1), (1, 40, 2), (33, 1, 3), (61, 97, 4), (321, 481, 5),
                                      (1080, 1920, 6)])
def test_contour_from_lab_bit_exact(H, W, seed):
    from paper_1903_07149_amd.maps import contour_from_lab
    img = synth.make_image(W, H, max(2, W * H // 4000), 10.0, seed)
    say("contour", H, W)
    got = host(contour_from_lab(dev(img.lab)))
    ref = OM.contour_prior(img.lab)
    assert (got == ref).all(), f"{int((got != ref).sum())} values differ"


def test_contour_of_constant_image_is_zero():
    from paper_1903_07149_amd.maps import contour_from_lab
    got = host(contour_from_lab(torch.full((20, 30, 3), 7.0, device="cuda")))
    assert (got == 0).all()


@pytest.mark.parametrize("W,H,k", [(160, 120, 48), (481, 321, 250)])
def test_fused_prior_equals_two_step(orc, W, H, k):
    """The prior fused into packing gives the run that the standalone prior
    map gives, and both equal the oracle run on the oracle's prior."""
    from paper_1903_07149_amd.maps import contour_from_lab
    from paper_1903_07149_amd.scalp import Scalp
    img = synth.make_image(W, H, 8, 10.0, 31)
    lab = dev(img.lab)
    say("fused prior", W, H, k)
    fused = Scalp(W, H, k, contour_source=CONTOUR_GRADIENT).run(lab, None)
    two = Scalp(W, H, k).run(lab, contour_from_lab(lab))
    for a, b in zip((fused.labels, fused.centers, fused.endpoints), (two.labels, two.centers, two.endpoints)):
        assert (host(a) == host(b)).all()
    ref = orc.run(img.lab, OM.contour_prior(img.lab), k, iterations=10, mode=orc.MEAN_FIXED)
    assert (host(fused.labels) == ref.labels).all()
    assert (host(fused.centers) == ref.centres).all()


def test_fused_prior_batched_per_image():
    """Batched packing normalises the prior per image."""
    from paper_1903_07149_amd.scalp import Scalp, ScalpBatch
    shapes = [(97, 61, 30), (160, 120, 48), (40, 300, 20)]
    imgs = [synth.make_image(w, h, 6, 10.0, 40 + i) for i, (w, h, _) in enumerate(shapes)]
    b = ScalpBatch(shapes, contour_source=CONTOUR_GRADIENT)
    lab = dev(np.concatenate([im.lab.reshape(-1, 3) for im in imgs]))
    say("fused prior batched")
    c, e, l, n = b.run(lab, None)
    l = host(l)
    for (p0, p1, H, W), (w, h, k), im in zip(b.pixel_slices(), shapes, imgs):
        r = Scalp(w, h, k, contour_source=CONTOUR_GRADIENT).run(dev(im.lab), None)
        assert (l[p0:p1].reshape(H, W) == host(r.labels)).all()


def test_gradient_prior_rejected_by_soft_and_null_contour_rejected():
    from paper_1903_07149_amd import _lib as L
    from paper_1903_07149_amd.scalp import Scalp
    from paper_1903_07149_amd.soft import SoftScalp
    eng = SoftScalp(32, 32, 16, 1, contour_source=CONTOUR_GRADIENT)
    with pytest.raises(L.ScalpError) as ei:
        eng.forward(torch.zeros((1, 32, 32, 3), device="cuda"), torch.zeros((1, 32, 32), device="cuda"))
    assert ei.value.code == L.SCALP_ERR_UNSUPPORTED
    with pytest.raises(L.ScalpError) as ei:
        Scalp(32, 32, 16).run(torch.zeros((32, 32, 3), device="cuda"), None)
    assert ei.value.code == L.SCALP_ERR_ARG


@pytest.mark.parametrize("tune", [dict(), dict(table_mode=1)])
def test_multiscale_boundary_map(orc, tune):
    """12 decompositions of the 481x321 image (6 to 600 superpixels) in one
    batch: every scale bit-exact against the oracle, and the boundary map
    bit-exact against the oracle's map of the oracle's labels (with both
    table modes of the assignment)."""
    from paper_1903_07149_amd.maps import MultiScale, scales
    img = synth.workload_image(synth.BSD_SHAPE)
    H, W = img.contour.shape
    ms = MultiScale(W, H, **tune)
    assert ms.ks == scales() and len(ms.ks) == 12 and ms.ks[0] == 6 and ms.ks[-1] == 600
    say("multiscale", W, H, ms.ks, tune)
    labels, bmap = ms.run(dev(img.lab), dev(img.contour))
    labels, bmap = host(labels), host(bmap)
    ref = []
    for s, k in enumerate(ms.ks):
        r = orc.run(img.lab, img.contour, k, iterations=10, mode=orc.MEAN_FIXED)
        assert (labels[s] == r.labels).all(), f"scale {k}"
        ref.append(r.labels)
    assert (bmap == OM.boundary_frequency(np.stack(ref))).all()
    # coarser scales have fewer boundary pixels
    nb = [(OM.boundary_frequency(l[None]) > 0).sum() for l in ref]
    assert nb[0] < nb[-1]
