"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/scalp.h declares, computes the same grid as the
oracle, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1903_07149_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scalp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scalp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in scalp.h but not exported"
    assert sorted(L.EXPORTED) == names


def test_grid_matches_oracle(orc):
    rng = np.random.default_rng(0)
    cases = [(481, 321, 250), (1920, 1080, 2000), (3840, 2160, 10000), (512, 512, 400),
             (1, 1, 1), (7, 1, 3), (1, 9, 9), (64, 48, 12), (100, 100, 10000), (33, 17, 561)]
    for _ in range(200):
        w, h = (int(v) for v in rng.integers(1, 3000, 2))
        cases.append((w, h, int(rng.integers(1, min(w * h, 20000) + 1))))
    for w, h, k in cases:
        g = L.make_grid(w, h, k)
        o = orc.grid(w, h, k)
        assert (g.nx, g.ny, g.num_sp) == (o.nx, o.ny, o.num_sp), (w, h, k)


def test_default_params():
    p = L.default_params()
    assert (p.m, p.lambda_, p.sigma, p.gamma) == (10.0, 0.5, 0.25, -1.0)
    assert (p.iterations, p.project, p.reuse_prepared) == (10, 1, 0)


def test_bad_arguments_are_rejected_on_host():
    lib = L.lib()
    g = L.make_grid(64, 48, 12)
    p = L.default_params()
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: validation fails first
    ws = L.workspace_bytes(g)
    assert ws >= 64 * 48 * 16 + 12 * 64
    for (w, h, k) in [(0, 5, 1), (5, 0, 1), (5, 5, 0), (5, 5, 26), (70000, 70000, 5)]:
        gg = L.Grid()
        assert lib.scalp_make_grid(w, h, k, ctypes.byref(gg)) == L.SCALP_ERR_ARG
    bad = L.Grid.from_buffer_copy(g)
    bad.nx += 1
    args = lambda gr, pr, wsz: (ctypes.byref(gr), ctypes.byref(pr), fake, fake, fake, fake,
                                fake, fake, wsz, None)
    assert lib.scalp_assign(*args(bad, p, ws)) == L.SCALP_ERR_ARG
    assert lib.scalp_assign(*args(g, p, ws - 1)) == L.SCALP_ERR_WORKSPACE
    assert lib.scalp_assign(ctypes.byref(g), ctypes.byref(p), fake, fake, fake, fake, fake,
                            None, ws, None) == L.SCALP_ERR_WORKSPACE
    for field, val in [("lambda_", 1.5), ("lambda_", -0.1), ("sigma", 0.0), ("m", -1.0),
                       ("iterations", -1), ("lds_pixels", 100000), ("wg_size", 128), ("wg_size", 768),
                       ("gamma", float("nan"))]:
        pp = L.default_params(**{field: val})
        assert lib.scalp_assign(*args(g, pp, ws)) == L.SCALP_ERR_ARG, field
    # null data pointers
    assert lib.scalp_assign(ctypes.byref(g), ctypes.byref(p), None, fake, fake, fake, fake,
                            fake, ws, None) == L.SCALP_ERR_ARG
    assert lib.scalp_run(ctypes.byref(g), ctypes.byref(p), fake, fake, fake, fake, fake, None,
                         fake, ws, None) == L.SCALP_ERR_ARG
    assert lib.scalp_update(ctypes.byref(g), ctypes.byref(p), fake, None, fake, fake, fake,
                            fake, ws, None) == L.SCALP_ERR_ARG
    assert lib.scalp_strerror(L.SCALP_ERR_WORKSPACE) == b"workspace missing or too small"


def test_batch_descriptors_must_be_concatenated():
    lib = L.lib()
    gs = [L.make_grid(40, 30, 12), L.make_grid(25, 60, 7)]
    d = (L.BatchDesc * 2)()
    d[0].pix_offset, d[0].sp_offset, d[0].grid = 0, 0, gs[0]
    d[1].pix_offset, d[1].sp_offset, d[1].grid = 1200, gs[0].num_sp, gs[1]
    assert lib.scalp_batch_workspace_bytes(d, 2) > 0
    d[1].pix_offset = 1201
    assert lib.scalp_batch_workspace_bytes(d, 2) == 0
    assert lib.scalp_batch_workspace_bytes(d, 0) == 0
