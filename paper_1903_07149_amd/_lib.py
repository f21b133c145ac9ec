"""ctypes binding of libscalp.so (include/scalp.h).

Argument marshalling only: every step of the clustering runs in the HIP
kernels of the library.  Tensors are torch CUDA (HIP) tensors; the stream is
torch's current stream unless one is given.  If the library has not been
built, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscalp.so")

SCALP_OK = 0
SCALP_ERR_ARG = -1
SCALP_ERR_WORKSPACE = -2
# SCALP_STATIC_SCRATCH_BYTES of include/scalp.h: the scratch of scalp_run_static
STATIC_SCRATCH_BYTES = 64 << 20
SCALP_ERR_HIP = -3
SCALP_ERR_UNSUPPORTED = -4

EXPORTED = [
    "scalp_default_params", "scalp_make_grid", "scalp_workspace_bytes", "scalp_prepare",
    "scalp_init_grid", "scalp_assign", "scalp_update", "scalp_assign_accumulate",
    "scalp_finalize", "scalp_run", "scalp_run_static", "scalp_graph_create",
    "scalp_graph_launch", "scalp_graph_destroy", "scalp_batch_workspace_bytes",
    "scalp_run_batched", "scalp_batched_graph_create", "scalp_soft_saved_bytes",
    "scalp_soft_workspace_bytes", "scalp_soft_forward", "scalp_soft_backward",
    "scalp_metrics_workspace_bytes", "scalp_metrics", "scalp_boundary_map",
    "scalp_contour_from_lab", "scalp_strerror",
]


class ScalpError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("k_requested", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("num_sp", ctypes.c_int32), ("r", ctypes.c_float)]

    def __repr__(self):
        return (f"Grid({self.width}x{self.height}, k={self.k_requested}, "
                f"{self.nx}x{self.ny}={self.num_sp})")


class Params(ctypes.Structure):
    _fields_ = [("m", ctypes.c_float), ("lambda_", ctypes.c_float), ("sigma", ctypes.c_float),
                ("gamma", ctypes.c_float), ("iterations", ctypes.c_int32),
                ("project", ctypes.c_int32), ("reuse_prepared", ctypes.c_int32),
                ("lds_pixels", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("assign_mode", ctypes.c_int32), ("contour_source", ctypes.c_int32),
                ("exact_pruning", ctypes.c_int32), ("persistent_blocks", ctypes.c_int32),
                ("table_mode", ctypes.c_int32)]


ASSIGN_GRID3X3 = 0
ASSIGN_WINDOW = 1
CONTOUR_INPUT = 0
CONTOUR_GRADIENT = 1


class BatchDesc(ctypes.Structure):
    _fields_ = [("pix_offset", ctypes.c_int64), ("sp_offset", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("grid", Grid)]


_lib = None
_P = ctypes.c_void_p
_SZ = ctypes.c_size_t


def lib() -> ctypes.CDLL:
    """The loaded HIP library.  Raises if it was not built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1903_07149_amd.build` "
                "(the SCALP path has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        gp = ctypes.POINTER(Grid)
        pp = ctypes.POINTER(Params)
        dp = ctypes.POINTER(BatchDesc)
        i32 = ctypes.c_int32
        f32 = ctypes.c_float
        sig = {
            "scalp_default_params": ([pp], ctypes.c_int),
            "scalp_make_grid": ([i32, i32, i32, gp], ctypes.c_int),
            "scalp_workspace_bytes": ([gp], _SZ),
            "scalp_prepare": ([gp, pp, _P, _P, _P, _SZ, _P], ctypes.c_int),
            "scalp_init_grid": ([gp, pp, _P, _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
            "scalp_assign": ([gp, pp, _P, _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
            "scalp_update": ([gp, pp, _P, _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
            "scalp_assign_accumulate": ([gp, pp, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
            "scalp_finalize": ([gp, pp, _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
            "scalp_run": ([gp, pp, _P, _P, _P, _P, _P, _P, _P, _SZ, _P], ctypes.c_int),
            "scalp_run_static": ([gp, pp, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
            "scalp_graph_create": ([gp, pp, _P, _P, _P, _P, _P, _SZ, ctypes.POINTER(_P)],
                                   ctypes.c_int),
            "scalp_graph_launch": ([_P, _P], ctypes.c_int),
            "scalp_graph_destroy": ([_P], ctypes.c_int),
            "scalp_batch_workspace_bytes": ([dp, i32], _SZ),
            "scalp_run_batched": ([dp, i32, pp, _P, _P, _P, _P, _P, _P, _P, _SZ, _P],
                                  ctypes.c_int),
            "scalp_batched_graph_create": ([dp, i32, pp, _P, _P, _P, _P, _P, _P, _P, _SZ,
                                            ctypes.POINTER(_P)], ctypes.c_int),
            "scalp_soft_saved_bytes": ([gp, i32, i32], _SZ),
            "scalp_soft_workspace_bytes": ([gp, i32], _SZ),
            "scalp_soft_forward": ([gp, pp, f32, i32, _P, _P, _P, _P, _P, _P, _SZ, _P],
                                   ctypes.c_int),
            "scalp_soft_backward": ([gp, pp, f32, i32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                     _SZ, _P], ctypes.c_int),
            "scalp_metrics_workspace_bytes": ([i32, i32, i32, i32], _SZ),
            "scalp_metrics": ([i32, i32, _P, i32, _P, i32, f32, _P, _P, _SZ, _P], ctypes.c_int),
            "scalp_boundary_map": ([i32, i32, _P, i32, _P, _P], ctypes.c_int),
            "scalp_contour_from_lab": ([i32, i32, _P, _P, _P, _SZ, _P], ctypes.c_int),
            "scalp_strerror": ([ctypes.c_int], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().scalp_strerror(int(code)).decode()
    except Exception:  # noqa: BLE001 - only used to format messages
        return "unknown"


def check(code: int, what: str) -> None:
    if code != SCALP_OK:
        raise ScalpError(code, what)


def make_grid(width: int, height: int, k: int) -> Grid:
    g = Grid()
    check(lib().scalp_make_grid(int(width), int(height), int(k), ctypes.byref(g)),
          "scalp_make_grid")
    return g


def apply_overrides(p: Params, overrides: dict) -> Params:
    names = {f[0] for f in Params._fields_}
    for key, val in overrides.items():
        key = "lambda_" if key in ("lam", "lambda") else key
        if key not in names:
            raise TypeError(f"unknown SCALP parameter {key!r}")
        setattr(p, key, val)
    return p


def default_params(**overrides) -> Params:
    p = Params()
    check(lib().scalp_default_params(ctypes.byref(p)), "scalp_default_params")
    return apply_overrides(p, overrides)


def workspace_bytes(g: Grid) -> int:
    return int(lib().scalp_workspace_bytes(ctypes.byref(g)))


def batch_workspace_bytes(descs) -> int:
    arr = (BatchDesc * len(descs))(*descs)
    return int(lib().scalp_batch_workspace_bytes(arr, len(descs)))


@dataclass
class Buffers:
    """Device tensors of one single-image problem."""
    centers: object
    endpoints: object
    labels: object
    counts: object
