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
    assert (p.exact_pruning, p.persistent_blocks, p.table_mode) == (1, 0, 0)


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


def test_mode_parameters_are_validated_on_host():
    lib = L.lib()
    g = L.make_grid(64, 48, 12)
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: validation fails first
    ws = L.workspace_bytes(g)
    args = lambda pr: (ctypes.byref(g), ctypes.byref(pr), fake, fake, fake, fake, fake, fake, ws,
                       None)
    for field, val in [("assign_mode", 2), ("assign_mode", -1), ("contour_source", 2),
                       ("contour_source", -1), ("exact_pruning", 2), ("exact_pruning", -1),
                       ("persistent_blocks", -1), ("persistent_blocks", 17),
                       ("table_mode", 2), ("table_mode", -1)]:
        pp = L.default_params(**{field: val})
        assert lib.scalp_assign(*args(pp)) == L.SCALP_ERR_ARG, (field, val)
    # a computed contour prior makes the contour pointer optional, a given one does not
    p = L.default_params()
    assert lib.scalp_prepare(ctypes.byref(g), ctypes.byref(p), fake, None, fake, ws,
                             None) == L.SCALP_ERR_ARG
    # the soft entry points support neither the window form nor a computed prior
    sw = lib.scalp_soft_workspace_bytes(ctypes.byref(g), 1)
    for over, code in [(dict(assign_mode=L.ASSIGN_WINDOW), L.SCALP_ERR_ARG),
                       (dict(contour_source=L.CONTOUR_GRADIENT), L.SCALP_ERR_UNSUPPORTED)]:
        pp = L.default_params(**over)
        assert lib.scalp_soft_forward(ctypes.byref(g), ctypes.byref(pp), ctypes.c_float(0.5), 1,
                                      fake, fake, fake, fake, fake, fake, sw, None) == code, over
    p = L.default_params()
    for batch in (0, 65536):
        assert lib.scalp_soft_forward(ctypes.byref(g), ctypes.byref(p), ctypes.c_float(0.5), batch,
                                      fake, fake, fake, fake, fake, fake, sw, None) == L.SCALP_ERR_ARG
    # 200 images of 8192 x 8192 with 2x2-pixel cells: 200 * 2^24 work items
    # do not fit a 32-bit grid (while 200 * 2^26 pixels are within the pixel limit)
    big = L.make_grid(8192, 8192, 8192 * 8192 // 4)
    assert big.num_sp == 4096 * 4096
    assert lib.scalp_soft_forward(ctypes.byref(big), ctypes.byref(p), ctypes.c_float(0.5), 200,
                                  fake, fake, fake, fake, fake, fake, 1 << 62, None) == L.SCALP_ERR_ARG
    with pytest.raises(TypeError):
        L.default_params(not_a_parameter=1)


def test_metrics_and_maps_validate_on_host():
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p(0x2000)
    assert lib.scalp_metrics_workspace_bytes(10, 10, 4, 3) > 0
    assert lib.scalp_metrics_workspace_bytes(0, 10, 4, 3) == 0
    assert lib.scalp_metrics_workspace_bytes(10, 10, 0, 3) == 0
    ws = lib.scalp_metrics_workspace_bytes(10, 10, 4, 3)
    f = ctypes.c_float
    assert lib.scalp_metrics(10, 10, fake, 4, fake, 3, f(2.0), out, fake, ws - 1,
                             None) == L.SCALP_ERR_WORKSPACE
    for eps in (0.0, -1.0, float("nan"), 100.0):
        assert lib.scalp_metrics(10, 10, fake, 4, fake, 3, f(eps), out, fake, ws,
                                 None) == L.SCALP_ERR_ARG, eps
    assert lib.scalp_metrics(10, 10, None, 4, fake, 3, f(2.0), out, fake, ws,
                             None) == L.SCALP_ERR_ARG
    assert lib.scalp_boundary_map(0, 5, fake, 2, out, None) == L.SCALP_ERR_ARG
    assert lib.scalp_boundary_map(5, 5, fake, 0, out, None) == L.SCALP_ERR_ARG
    assert lib.scalp_boundary_map(5, 5, None, 2, out, None) == L.SCALP_ERR_ARG
    assert lib.scalp_contour_from_lab(5, 5, fake, out, fake, 4, None) == L.SCALP_ERR_WORKSPACE
    assert lib.scalp_contour_from_lab(5, 5, fake, out, fake, 4095, None) == L.SCALP_ERR_WORKSPACE
    assert lib.scalp_contour_from_lab(5, 0, fake, out, fake, 8, None) == L.SCALP_ERR_ARG
    assert lib.scalp_contour_from_lab(5, 5, None, out, fake, 8, None) == L.SCALP_ERR_ARG


def test_static_run_limits_are_checked_on_host():
    """scalp_run_static rejects, before any HIP call, a workspace larger than
    its scratch and a request to reuse a packed image."""
    lib = L.lib()
    z = ctypes.c_void_p(0x1000)             # never dereferenced: validation fails first
    p = L.default_params()
    big = L.make_grid(3840, 2160, 10000)
    assert L.workspace_bytes(big) > L.STATIC_SCRATCH_BYTES
    assert lib.scalp_run_static(ctypes.byref(big), ctypes.byref(p), z, z, z, z, z, z,
                                None) == L.SCALP_ERR_WORKSPACE
    hd = L.make_grid(1920, 1080, 2000)
    assert L.workspace_bytes(hd) <= L.STATIC_SCRATCH_BYTES
    p.reuse_prepared = 1
    assert lib.scalp_run_static(ctypes.byref(hd), ctypes.byref(p), z, z, z, z, z, z,
                                None) == L.SCALP_ERR_ARG
    p.reuse_prepared = 0
    assert lib.scalp_run_static(ctypes.byref(hd), ctypes.byref(p), z, z, None, z, z, z,
                                None) == L.SCALP_ERR_ARG
