"""MI355X (gfx950) implementation of the SCALP clustering path
("Superpixels with Contour Adherence using Linear Path", arXiv 1903.07149).

The compute path is libscalp.so (HIP kernels behind a C ABI, include/scalp.h);
this package holds its ctypes binding, torch wrappers and the seeded
synthetic-input generator.
"""
from ._lib import Grid, Params, ScalpError, default_params, make_grid  # noqa: F401

__all__ = ["Grid", "Params", "ScalpError", "default_params", "make_grid"]
