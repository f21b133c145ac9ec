"""GPU quality metrics (scalp_metrics) against the numpy definitions, and the
distance ablation of Sec. III-B on synthetic ground truth."""
import numpy as np
import pytest

from oracle import metrics as M
from paper_1903_07149_amd import synth
from gpu_util import dev, host, needs_gpu, say, torch

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.mark.parametrize("eps", [2.0, 1.0, 3.5, 5.0])
@pytest.mark.parametrize("H,W,K,R,seed", [(37, 53, 9, 5, 1), (128, 96, 40, 12, 2), (1, 70, 4, 3, 3),
                                          (64, 1, 2, 2, 4)])
def test_metrics_match_definitions(H, W, K, R, seed, eps):
    from paper_1903_07149_amd.metrics import metrics
    rng = np.random.default_rng(seed)
    # blocky label maps, so that boundaries are sparse and structured
    sp = np.kron(rng.integers(0, K, (H // 4 + 1, W // 4 + 1)), np.ones((4, 4)))[:H, :W]
    gt = np.kron(rng.integers(0, R, (H // 6 + 1, W // 6 + 1)), np.ones((6, 6)))[:H, :W]
    sp, gt = sp.astype(np.int32), gt.astype(np.int32)
    say("metrics", H, W, K, R, eps)
    got = metrics(dev(sp), dev(gt), num_sp=K, num_regions=R, epsilon=eps)
    ref = M.all_metrics(sp, gt, eps)
    assert got["br"] == ref["br"] and got["asa"] == ref["asa"] and got["ue"] == ref["ue"]
    assert abs(got["co"] - ref["co"]) <= 1e-12 * max(1.0, ref["co"])
    assert got["gt_boundary"] == int(M.boundary(gt).sum())
    assert got["sp_boundary"] == int(M.boundary(sp).sum())


@pytest.mark.parametrize("eps", [17.5, 40.25, 63.9, 64.0])
def test_boundary_recall_far_and_across_words(eps):
    """Sparse superpixel boundaries (two vertical cuts, one short horizontal
    one) and ground-truth boundaries at many distances: recall then hinges on
    the search reaching across 64-pixel words and many rows."""
    from paper_1903_07149_amd.metrics import metrics
    H, W = 90, 333
    sp = np.zeros((H, W), np.int32)
    sp[:, 150:] = 1
    sp[:, 290:] = 2
    sp[70:, 20:60] = 3
    rng = np.random.default_rng(7)
    gt = np.zeros((H, W), np.int32)
    for v, c in enumerate(sorted(rng.choice(np.arange(1, W), 9, replace=False)), start=1):
        gt[:, c:] = v
    gt[rng.integers(0, H):, :40] += 10
    say("metrics far", H, W, eps)
    got = metrics(dev(sp), dev(gt), num_sp=4, num_regions=int(gt.max()) + 1, epsilon=eps)
    ref = M.all_metrics(sp, gt, eps)
    assert got["br"] == ref["br"]
    assert got["gt_boundary"] == int(M.boundary(gt).sum())
    assert got["sp_boundary"] == int(M.boundary(sp).sum())


def test_metrics_with_more_pairs_than_the_lds_table():
    """Per-pixel random labels and regions: a 256-column block of a few rows
    meets far more than 512 distinct (superpixel, region) pairs, so most of
    them overflow the workgroup's LDS pair table and go to global memory
    directly."""
    from paper_1903_07149_amd.metrics import metrics
    rng = np.random.default_rng(23)
    H, W, K, R = 1100, 2048, 5000, 300          # blocks of 256 columns x 8 rows
    sp = rng.integers(0, K, (H, W)).astype(np.int32)
    gt = rng.integers(0, R, (H, W)).astype(np.int32)
    say("metrics overflow", H, W, K, R)
    got = metrics(dev(sp), dev(gt), num_sp=K, num_regions=R, epsilon=2.0)
    ref = M.all_metrics(sp, gt, 2.0)
    assert got["br"] == ref["br"] and got["asa"] == ref["asa"] and got["ue"] == ref["ue"]
    assert abs(got["co"] - ref["co"]) <= 1e-12 * max(1.0, ref["co"])


def test_boundary_recall_at_the_tolerance():
    """Offsets at exactly epsilon do not count (the oracle's closed-form case)."""
    from paper_1903_07149_amd.metrics import metrics
    g = np.zeros((30, 30), np.int32)
    g[10, 10] = 1
    s = np.zeros_like(g)
    s[14, 14] = 1
    got = metrics(dev(s), dev(g), num_sp=2, num_regions=2, epsilon=5.0)
    assert got["br"] == 2 / 5 == M.boundary_recall(s, g, 5.0)


def test_metrics_of_a_run_and_ablation():
    """Metrics of SCALP label maps against the Voronoi ground truth, for the four
    distance settings of Sec. III-B: SLIC (lambda = 1, gamma = 0), + path colour
    (lambda = 0.5), + contour (gamma = 2r), and full SCALP."""
    from paper_1903_07149_amd.metrics import metrics
    from paper_1903_07149_amd.scalp import Scalp
    img = synth.workload_image(synth.BSD_SHAPE)
    H, W = img.contour.shape
    lab, con, gt = dev(img.lab), dev(img.contour), dev(img.gt)
    rows = {}
    for name, kw in [("slic", dict(lam=1.0, gamma=0.0)), ("path_colour", dict(lam=0.5, gamma=0.0)),
                     ("contour", dict(lam=1.0)), ("scalp", dict())]:
        s = Scalp(W, H, 250, **kw)
        say("ablation", name)
        r = s.run(lab, con)
        m = metrics(r.labels, gt, num_sp=s.K)
        ref = M.all_metrics(host(r.labels), img.gt)
        assert m["br"] == ref["br"] and m["asa"] == ref["asa"] and m["ue"] == ref["ue"]
        assert abs(m["co"] - ref["co"]) <= 1e-12
        rows[name] = m
        print(name, {k: round(v, 4) for k, v in m.items()})
    # Sec. III-B/III-C: the path terms make superpixels more homogeneous and more
    # compact than SLIC's (BR saturates at 1 here: SLIC's noisy boundaries cover
    # nearly every pixel, so it is not compared)
    assert rows["scalp"]["ue"] < rows["slic"]["ue"]
    assert rows["scalp"]["asa"] > rows["slic"]["asa"]
    assert rows["scalp"]["co"] > rows["slic"]["co"]
    assert rows["scalp"]["sp_boundary"] < rows["slic"]["sp_boundary"]


def test_ablation_with_a_finer_ground_truth():
    """The distance ablation of Sec. III-B where boundary recall does not
    saturate: 300 ground-truth regions against 250 superpixels (481x321, noise
    sigma 10), so superpixel boundaries cannot reach every region boundary.
    The paper compares the settings by precision-recall; here boundary recall
    (GT boundary pixels with a superpixel boundary pixel closer than 2),
    boundary precision (the same measure with the two maps swapped) and their
    F-measure.  As in Sec. III-B: the contour term raises recall (over SLIC,
    and over the path colour alone), and each term raises the F-measure over
    SLIC's, full SCALP scoring best."""
    from paper_1903_07149_amd.metrics import metrics
    from paper_1903_07149_amd.scalp import Scalp
    img = synth.make_image(481, 321, 300, 10.0, 1)
    H, W = img.contour.shape
    R = int(img.gt.max()) + 1
    lab, con, gt = dev(img.lab), dev(img.contour), dev(img.gt)
    rows = {}
    for name, kw in [("slic", dict(lam=1.0, gamma=0.0)), ("path_colour", dict(lam=0.5, gamma=0.0)),
                     ("contour", dict(lam=1.0)), ("scalp", dict())]:
        s = Scalp(W, H, 250, **kw)
        say("fine-gt ablation", name)
        r = s.run(lab, con)
        m = metrics(r.labels, gt, num_sp=s.K, num_regions=R)
        bp = metrics(gt, r.labels, num_sp=R, num_regions=s.K)["br"]   # precision
        assert m["br"] == M.boundary_recall(host(r.labels), img.gt, 2.0)
        assert bp == M.boundary_recall(img.gt, host(r.labels), 2.0)
        f = 2 * bp * m["br"] / (bp + m["br"])
        rows[name] = dict(br=m["br"], bp=bp, f=f)
        print(name, {k: round(v, 4) for k, v in rows[name].items()})
    assert all(v["br"] < 0.99 for v in rows.values())            # not saturated
    assert rows["contour"]["br"] > rows["slic"]["br"]
    assert rows["scalp"]["br"] > rows["path_colour"]["br"]
    assert rows["path_colour"]["f"] > rows["slic"]["f"]
    assert rows["contour"]["f"] > rows["slic"]["f"]
    assert rows["scalp"]["f"] > max(rows["slic"]["f"], rows["path_colour"]["f"],
                                    rows["contour"]["f"])


def test_reusable_metrics_call_matches():
    """metrics.Metrics (workspace allocated once, result left on the device)
    gives what metrics() gives, on repeated calls."""
    from paper_1903_07149_amd.metrics import Metrics, metrics
    rng = np.random.default_rng(11)
    H, W, K, R = 70, 90, 12, 5
    sp = np.kron(rng.integers(0, K, (H // 5 + 1, W // 5 + 1)), np.ones((5, 5)))[:H, :W].astype(np.int32)
    gt = np.kron(rng.integers(0, R, (H // 7 + 1, W // 7 + 1)), np.ones((7, 7)))[:H, :W].astype(np.int32)
    ref = metrics(dev(sp), dev(gt), num_sp=K, num_regions=R, epsilon=2.0)
    mk = Metrics(W, H, K, R, epsilon=2.0)
    for _ in range(3):
        v = host(mk.run(dev(sp), dev(gt))).tolist()
        assert v[:4] == [ref["br"], ref["asa"], ref["ue"], ref["co"]]
        assert int(v[4]) == ref["gt_boundary"] and int(v[5]) == ref["sp_boundary"]
