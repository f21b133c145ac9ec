"""ctypes wrapper over the plain C oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.  The library is
built by :func:`build` with gcc (no contraction, no fast-math), so its FP32
arithmetic follows IEEE single precision operation by operation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ["scalp_oracle.c", "scalp_soft_oracle.c"]
LIB_PATH = os.path.join(_HERE, "liboracle.so")
# A test may point the wrapper at another build of the oracle sources (the
# mutation test plants mistakes in a temporary copy to prove the pins fail).
_LIB_OVERRIDE = os.environ.get("SCALP_ORACLE_LIB")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fexcess-precision=standard",
          "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function"]

MEAN_PLAIN = 0
MEAN_FIXED = 1


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (always recompiles)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            _lib = ctypes.CDLL(_LIB_OVERRIDE)
            _declare(_lib)
            return _lib
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_i = ctypes.c_int
_l = ctypes.c_long
_f = ctypes.c_float
_d = ctypes.c_double
_p = ctypes.c_void_p


def _declare(L):
    L.orc_grid_r.argtypes = [_i, _i, _i]; L.orc_grid_r.restype = _d
    L.orc_grid.argtypes = [_i, _i, _i, _p, _p]; L.orc_grid.restype = _i
    L.orc_spatial_weight.argtypes = [_i, _i, _i, _f]; L.orc_spatial_weight.restype = _f
    L.orc_default_gamma.argtypes = [_i, _i, _i]; L.orc_default_gamma.restype = _f
    L.orc_wmap.argtypes = [_p, _l, _f, _p]; L.orc_wmap.restype = None
    L.orc_path.argtypes = [_i, _i, _i, _i, _p, _p]; L.orc_path.restype = _i
    L.orc_distance.argtypes = [_i, _i, _p, _p, _f, _f, _f, _i, _i, _p, _i, _i]
    L.orc_distance.restype = _f
    L.orc_assign.argtypes = [_i, _i, _i, _i, _p, _p, _p, _p, _f, _f, _f, _p, _p, _p]
    L.orc_assign.restype = None
    L.orc_update.argtypes = [_i, _i, _i, _p, _p, _i, _p, _p]; L.orc_update.restype = None
    L.orc_round_endpoints.argtypes = [_i, _i, _i, _p, _p]; L.orc_round_endpoints.restype = None
    L.orc_project.argtypes = [_i, _i, _i, _p, _p, _p, _p]; L.orc_project.restype = _i
    L.orc_init_grid.argtypes = [_i, _i, _i, _i, _p, _i, _p, _p, _p]
    L.orc_init_grid.restype = None
    L.orc_run.argtypes = [_i, _i, _i, _p, _p, _f, _f, _f, _f, _i, _i, _i, _p, _p, _p, _p]
    L.orc_run.restype = _l
    L.orc_window_radius.argtypes = [_i, _i, _i]; L.orc_window_radius.restype = _i
    L.orc_assign_window.argtypes = [_i, _i, _i, _i, _p, _p, _p, _p, _f, _f, _f, _p, _p]
    L.orc_assign_window.restype = None
    L.orc_run_window.argtypes = [_i, _i, _i, _p, _p, _f, _f, _f, _f, _i, _i, _i, _p, _p, _p,
                                 _p]
    L.orc_run_window.restype = _l
    L.orc_set_threads.argtypes = [_i]; L.orc_set_threads.restype = None
    L.orc_max_threads.argtypes = []; L.orc_max_threads.restype = _i
    L.orc_distance_ab.argtypes = [_i, _i, _p, _p, _f, _f, _f, _i, _i, _p, _i, _i, _p, _p, _p]
    L.orc_distance_ab.restype = _f
    L.orc_soft_forward.argtypes = [_i, _i, _i, _i, _p, _p, _d, _d, _d, _d, _d, _i, _i, _p, _p,
                                   _p]
    L.orc_soft_forward.restype = _i
    L.orc_soft_backward.argtypes = [_i, _i, _i, _i, _p, _p, _d, _d, _d, _d, _d, _i, _i, _p,
                                    _p, _p, _p]
    L.orc_soft_backward.restype = _i
    L.orc_soft_backward_ex.argtypes = [_i, _i, _i, _i, _p, _p, _d, _d, _d, _d, _d, _i, _i, _p,
                                       _p, _p, _p, _i, _i, _p]
    L.orc_soft_backward_ex.restype = _i


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass(frozen=True)
class Grid:
    width: int
    height: int
    k: int
    nx: int
    ny: int

    @property
    def num_sp(self) -> int:
        return self.nx * self.ny

    @property
    def r(self) -> float:
        return lib().orc_grid_r(self.width, self.height, self.k)


def grid(width: int, height: int, k: int) -> Grid:
    nx = ctypes.c_int()
    ny = ctypes.c_int()
    K = lib().orc_grid(width, height, k, ctypes.byref(nx), ctypes.byref(ny))
    if K < 0:
        raise ValueError(f"invalid grid {width}x{height} k={k}")
    return Grid(width, height, k, nx.value, ny.value)


def spatial_weight(g: Grid, m: float = 10.0) -> float:
    return float(lib().orc_spatial_weight(g.width, g.height, g.k, m))


def default_gamma(g: Grid) -> float:
    return float(lib().orc_default_gamma(g.width, g.height, g.k))


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def wmap(contour: np.ndarray, sigma: float = 0.25) -> np.ndarray:
    c = _f32(contour)
    w = np.empty_like(c)
    lib().orc_wmap(_ptr(c), c.size, sigma, _ptr(w))
    return w


def path(x: int, y: int, cx: int, cy: int) -> np.ndarray:
    n = max(abs(cx - x), abs(cy - y))
    qx = np.empty(n + 1, np.int32)
    qy = np.empty(n + 1, np.int32)
    cnt = lib().orc_path(x, y, cx, cy, _ptr(qx), _ptr(qy))
    assert cnt == n + 1
    return np.stack([qx, qy], axis=1)


def distance(lab, w, x, y, centre, endpoint, lam=0.5, gamma=50.0, spw=0.1) -> float:
    lab = _f32(lab)
    w = _f32(w)
    H, W = w.shape
    c = _f32(centre)
    return float(lib().orc_distance(W, H, _ptr(lab), _ptr(w), lam, gamma, spw, int(x), int(y),
                                    _ptr(c), int(endpoint[0]), int(endpoint[1])))


def assign(g: Grid, lab, w, centres, endpoints, lam=0.5, gamma=None, spw=None,
           m: float = 10.0):
    """One assignment pass from fixed centres/endpoints.
    Returns (labels int32[H][W], best D float32[H][W], path samples)."""
    lab = _f32(lab)
    w = _f32(w)
    centres = _f32(centres)
    endpoints = _i32(endpoints)
    if gamma is None:
        gamma = default_gamma(g)
    if spw is None:
        spw = spatial_weight(g, m)
    labels = np.empty((g.height, g.width), np.int32)
    best = np.empty((g.height, g.width), np.float32)
    samples = ctypes.c_long()
    lib().orc_assign(g.width, g.height, g.nx, g.ny, _ptr(lab), _ptr(w), _ptr(centres),
                     _ptr(endpoints), lam, gamma, spw, _ptr(labels), _ptr(best),
                     ctypes.byref(samples))
    return labels, best, samples.value


def window_radius(g: Grid) -> int:
    return int(lib().orc_window_radius(g.width, g.height, g.k))


def assign_window(g: Grid, lab, w, centres, endpoints, labels, lam=0.5, gamma=None, spw=None,
                  m: float = 10.0, R: int | None = None):
    """Cluster-centric assignment of Algorithm 1 (windows of half-width R around the
    rounded barycenters).  `labels` holds the previous labels (kept where no window
    covers a pixel).  Returns (labels, best D; +inf where uncovered)."""
    lab = _f32(lab)
    w = _f32(w)
    centres = _f32(centres)
    endpoints = _i32(endpoints)
    out = _i32(labels).copy()
    if gamma is None:
        gamma = default_gamma(g)
    if spw is None:
        spw = spatial_weight(g, m)
    if R is None:
        R = window_radius(g)
    best = np.empty((g.height, g.width), np.float32)
    lib().orc_assign_window(g.width, g.height, g.num_sp, R, _ptr(lab), _ptr(w), _ptr(centres),
                            _ptr(endpoints), lam, gamma, spw, _ptr(out), _ptr(best))
    return out, best


def update(g: Grid, lab, labels, centres, mode: int = MEAN_PLAIN):
    """Returns (new centres float32[K][5], counts int32[K])."""
    lab = _f32(lab)
    labels = _i32(labels)
    out = _f32(centres).copy()
    counts = np.empty(g.num_sp, np.int32)
    lib().orc_update(g.width, g.height, g.num_sp, _ptr(lab), _ptr(labels), mode, _ptr(out),
                     _ptr(counts))
    return out, counts


def round_endpoints(g: Grid, centres) -> np.ndarray:
    centres = _f32(centres)
    ep = np.empty((g.num_sp, 2), np.int32)
    lib().orc_round_endpoints(g.width, g.height, g.num_sp, _ptr(centres), _ptr(ep))
    return ep


def project(g: Grid, labels, centres, counts, endpoints):
    """Returns (new endpoints int32[K][2], number moved)."""
    labels = _i32(labels)
    centres = _f32(centres)
    counts = _i32(counts)
    ep = _i32(endpoints).copy()
    moved = lib().orc_project(g.width, g.height, g.num_sp, _ptr(labels), _ptr(centres),
                              _ptr(counts), _ptr(ep))
    return ep, moved


def init_grid(g: Grid, lab, mode: int = MEAN_PLAIN):
    """Returns (centres float32[K][5], endpoints int32[K][2], labels int32[H][W])."""
    lab = _f32(lab)
    centres = np.empty((g.num_sp, 5), np.float32)
    ep = np.empty((g.num_sp, 2), np.int32)
    labels = np.empty((g.height, g.width), np.int32)
    lib().orc_init_grid(g.width, g.height, g.nx, g.ny, _ptr(lab), mode, _ptr(centres),
                        _ptr(ep), _ptr(labels))
    return centres, ep, labels


@dataclass
class RunResult:
    labels: np.ndarray
    centres: np.ndarray
    endpoints: np.ndarray
    counts: np.ndarray
    samples: int


def run(lab, contour, k: int, iterations: int = 10, m: float = 10.0, lam: float = 0.5,
        sigma: float = 0.25, gamma: float = -1.0, project: bool = True,
        mode: int = MEAN_PLAIN) -> RunResult:
    lab = _f32(lab)
    contour = _f32(contour)
    H, W = contour.shape
    g = grid(W, H, k)
    centres = np.empty((g.num_sp, 5), np.float32)
    ep = np.empty((g.num_sp, 2), np.int32)
    labels = np.empty((H, W), np.int32)
    counts = np.zeros(g.num_sp, np.int32)
    s = lib().orc_run(W, H, k, _ptr(lab), _ptr(contour), m, lam, sigma, gamma, iterations,
                      int(project), mode, _ptr(centres), _ptr(ep), _ptr(labels), _ptr(counts))
    if s < 0:
        raise ValueError("oracle run rejected its arguments")
    return RunResult(labels, centres, ep, counts, int(s))


def run_window(lab, contour, k: int, iterations: int = 10, m: float = 10.0, lam: float = 0.5,
               sigma: float = 0.25, gamma: float = -1.0, project: bool = True,
               mode: int = MEAN_PLAIN) -> RunResult:
    """Whole run with the window assignment of Algorithm 1."""
    lab = _f32(lab)
    contour = _f32(contour)
    H, W = contour.shape
    g = grid(W, H, k)
    centres = np.empty((g.num_sp, 5), np.float32)
    ep = np.empty((g.num_sp, 2), np.int32)
    labels = np.empty((H, W), np.int32)
    counts = np.zeros(g.num_sp, np.int32)
    s = lib().orc_run_window(W, H, k, _ptr(lab), _ptr(contour), m, lam, sigma, gamma, iterations,
                             int(project), mode, _ptr(centres), _ptr(ep), _ptr(labels),
                             _ptr(counts))
    if s < 0:
        raise ValueError("oracle run rejected its arguments")
    return RunResult(labels, centres, ep, counts, 0)


def soft_forward(lab, contour, k: int, iterations: int = 5, m: float = 10.0,
                 lam: float = 0.5, sigma: float = 0.25, gamma: float = -1.0, T: float = 0.5,
                 d32: bool = False):
    """lab float32[B][H][W][3], contour float32[B][H][W].
    Returns (theta f64[iters+1][B][K][5], q f64[iters][B][H][W][9], z f64[iters][B][K]).
    d32: the FP32-distance precision mode (see scalp_soft_oracle.c)."""
    lab = _f32(lab)
    contour = _f32(contour)
    B, H, W = contour.shape
    g = grid(W, H, k)
    K = g.num_sp
    theta = np.zeros((iterations + 1, B, K, 5))
    q = np.zeros((iterations, B, H, W, 9))
    z = np.zeros((iterations, B, K))
    rc = lib().orc_soft_forward(B, W, H, k, _ptr(lab), _ptr(contour), m, lam, sigma, gamma, T,
                                iterations, int(d32), _ptr(theta), _ptr(q), _ptr(z))
    if rc != 0:
        raise ValueError("oracle soft forward rejected its arguments")
    return theta, q, z


def soft_backward(lab, contour, k: int, gq, gtheta, iterations: int = 5, m: float = 10.0,
                  lam: float = 0.5, sigma: float = 0.25, gamma: float = -1.0, T: float = 0.5,
                  d32: bool = False, qcut: bool = False, r32: bool = False, bound: bool = False):
    """Gradient of <gq, Q_T> + <gtheta, Theta_T>.  Returns (glab f64[B][H][W][3],
    gcontour f64[B][H][W]), plus, with bound=True, a dict of the error bound of
    an FP32 evaluation (see scalp_soft_oracle.c): for "lab" and "contour" each,
    (E, Md); an FP32 evaluation errs by at most 2^-24 E + Md per element (first
    order), Md being what leaving out the slots with Q < 2^-24 can change.
    qcut: leave out the slots whose Q is below 2^-24; r32: round every
    intermediate result to FP32 (both test infrastructure for the bound)."""
    lab = _f32(lab)
    contour = _f32(contour)
    B, H, W = contour.shape
    gq = _f64(gq)
    gtheta = _f64(gtheta)
    glab = np.zeros((B, H, W, 3))
    gc = np.zeros((B, H, W))
    arrays = None
    bnd_ptr = None
    if bound:
        arrays = [np.zeros((B, H, W, 3)) for _ in range(2)] + [np.zeros((B, H, W)) for _ in range(2)]
        table = (ctypes.c_void_p * 4)(*[_ptr(a) for a in arrays])
        bnd_ptr = ctypes.cast(table, ctypes.c_void_p).value
    rc = lib().orc_soft_backward_ex(B, W, H, k, _ptr(lab), _ptr(contour), m, lam, sigma, gamma, T,
                                    iterations, int(d32), _ptr(gq), _ptr(gtheta), _ptr(glab),
                                    _ptr(gc), int(qcut), int(r32), bnd_ptr)
    if rc != 0:
        raise ValueError("oracle soft backward rejected its arguments")
    if not bound:
        return glab, gc
    return glab, gc, {"lab": tuple(arrays[:2]), "contour": tuple(arrays[2:])}
