"""scalp_run_static, the allocation-free variant of scalp_run (its workspace is
the library's own device scratch), through the C ABI against scalp_run itself:
labels, centres, endpoints and counts bit-identical, on two calls in a row
with the second on a smaller image (what the first left in the shared
scratch must not leak into it), in the grid form and the window form."""
import ctypes

import numpy as np
import pytest

from paper_1903_07149_amd import _lib as L
from paper_1903_07149_amd import synth
from gpu_util import dev, host, needs_gpu, say, torch

pytestmark = [pytest.mark.gpu, needs_gpu]


def _both(W, H, k, regions, seed, **over):
    from paper_1903_07149_amd.scalp import Scalp
    img = synth.make_image(W, H, regions, 10.0, seed)
    s = Scalp(W, H, k, **over)
    lab, con = dev(img.lab), dev(img.contour)
    ref = s.run(lab, con)
    out = s.new_state()
    torch.cuda.synchronize()
    got = s.run_static(lab, con, out=out)
    return [host(t) for t in (ref.labels, ref.centers, ref.endpoints, ref.counts)], \
           [host(t) for t in (got.labels, got.centers, got.endpoints, got.counts)]


def test_static_equals_run_twice_second_smaller():
    mode = L.ASSIGN_WINDOW
    for W, H, k, regions, seed, over in [(1920, 1080, 2000, 400, 2, {}),
                                         (481, 321, 250, 40, 1, {}),
                                         (300, 200, 60, 12, 7, {"assign_mode": mode})]:
        say("scalp_run_static", W, H, k, over)
        ref, got = _both(W, H, k, regions, seed, **over)
        for a, b, name in zip(ref, got, ("labels", "centers", "endpoints", "counts")):
            assert np.array_equal(a, b), (W, H, name)


def test_static_rejects_what_does_not_fit():
    g = L.make_grid(3840, 2160, 10000)
    assert L.workspace_bytes(g) > L.STATIC_SCRATCH_BYTES
    p = L.default_params()
    z = ctypes.c_void_p(0x1000)
    rc = L.lib().scalp_run_static(ctypes.byref(g), ctypes.byref(p), z, z, z, z, z, z, None)
    assert rc == L.SCALP_ERR_WORKSPACE
