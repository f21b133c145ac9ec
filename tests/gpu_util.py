"""Helpers shared by the GPU tests (device plumbing only)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU visible")


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def say(*msg):
    """Names the case before a GPU step, so a fault still identifies it."""
    print("[gpu-case]", *msg, flush=True)
    sys.stdout.flush()


def perturbed_state(orc, g, lab, seed, jitter=3.0, colour=10.0):
    """Oracle grid initialisation moved by a seeded perturbation (CPU only)."""
    centres, ep, _ = orc.init_grid(g, lab, mode=orc.MEAN_FIXED)
    rng = np.random.default_rng(seed)
    c = centres.copy()
    c[:, 0:3] += rng.normal(0, colour, (g.num_sp, 3)).astype(np.float32)
    c[:, 3] = np.clip(c[:, 3] + rng.uniform(-jitter, jitter, g.num_sp), 0, g.width - 1)
    c[:, 4] = np.clip(c[:, 4] + rng.uniform(-jitter, jitter, g.num_sp), 0, g.height - 1)
    c = c.astype(np.float32)
    return c, orc.round_endpoints(g, c)
