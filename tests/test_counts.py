"""The algorithmic sample count used for throughput/roofline figures equals the
number of path samples the oracle evaluates."""
import numpy as np

from paper_1903_07149_amd import counts, synth


def test_sample_count_matches_oracle(orc):
    for (W, H, k, seed) in [(97, 61, 30, 1), (160, 120, 48, 2), (50, 1, 5, 3)]:
        lab, con = synth.random_lab(W, H, seed)
        g = orc.grid(W, H, k)
        c, e, _ = orc.init_grid(g, lab)
        rng = np.random.default_rng(seed)
        c[:, 3] = np.clip(c[:, 3] + rng.uniform(-3, 3, g.num_sp), 0, W - 1)
        c[:, 4] = np.clip(c[:, 4] + rng.uniform(-3, 3, g.num_sp), 0, H - 1)
        e = orc.round_endpoints(g, c)
        _, _, samples = orc.assign(g, lab, orc.wmap(con), c, e)
        w = counts.pass_work(W, H, g.nx, g.ny, e)
        assert w["samples"] == samples
        assert w["flops"] == 10 * samples + 16 * w["candidates"]


def test_window_sample_count_brute_force(orc):
    """The window form's sample count, summed per cluster over its window, equals
    the count summed per pixel over the clusters whose window contains it."""
    for (W, H, k, seed) in [(37, 23, 12, 4), (60, 41, 30, 5)]:
        lab, con = synth.random_lab(W, H, seed)
        g = orc.grid(W, H, k)
        c, e, _ = orc.init_grid(g, lab)
        rng = np.random.default_rng(seed)
        c[:, 3] = np.clip(c[:, 3] + rng.uniform(-4, 4, g.num_sp), 0, W - 1)
        c[:, 4] = np.clip(c[:, 4] + rng.uniform(-4, 4, g.num_sp), 0, H - 1)
        e = orc.round_endpoints(g, c)
        R = orc.window_radius(g)
        w = counts.window_work(W, H, R, c, e)
        cx = [min(max(int(np.floor(np.float32(c[q, 3]) + np.float32(0.5))), 0), W - 1) for q in range(g.num_sp)]
        cy = [min(max(int(np.floor(np.float32(c[q, 4]) + np.float32(0.5))), 0), H - 1) for q in range(g.num_sp)]
        samples = cands = 0
        for y in range(H):
            for x in range(W):
                for q in range(g.num_sp):
                    if abs(x - cx[q]) <= R and abs(y - cy[q]) <= R:
                        samples += max(abs(int(e[q, 0]) - x), abs(int(e[q, 1]) - y)) + 1
                        cands += 1
        assert (w["samples"], w["candidates"]) == (samples, cands)


def test_soft_backward_count_brute_force(orc):
    """The soft backward's re-walked samples, summed slot-plane by slot-plane,
    equal a per-pixel loop over the walked pairs with the oracle's own path
    length (its path from the pixel to the slot's endpoint)."""
    rng = np.random.default_rng(12)
    for (W, H, k) in [(23, 17, 6), (40, 9, 8)]:
        g = orc.grid(W, H, k)
        ep = np.stack([rng.integers(0, W, g.num_sp), rng.integers(0, H, g.num_sp)], 1)
        walked = rng.random((9, H, W)) < 0.4
        w = counts.soft_backward_work(W, H, g.nx, g.ny, ep, walked)
        samples = pairs = 0
        for y in range(H):
            for x in range(W):
                ci, cj = (y * g.ny) // H, (x * g.nx) // W
                for j in range(9):
                    ii, jj = ci + j // 3 - 1, cj + j % 3 - 1
                    if 0 <= ii < g.ny and 0 <= jj < g.nx and walked[j, y, x]:
                        kk = ii * g.nx + jj
                        samples += len(orc.path(x, y, int(ep[kk, 0]), int(ep[kk, 1])))
                        pairs += 1
        assert (w["samples"], w["pairs"]) == (samples, pairs)
        assert w["flops"] == 13 * samples + 14 * pairs + 171 * W * H
