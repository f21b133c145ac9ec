"""Torch-facing wrappers of the SCALP C ABI (device memory and streams only).

Every function validates shapes/dtypes/devices, then hands raw device
pointers and torch's current HIP stream to libscalp.so.  No arithmetic of the
method happens here.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L
from ._lib import BatchDesc, Grid, Params, check, default_params, make_grid


def _p(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(stream: torch.cuda.Stream | None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need(t: torch.Tensor, shape, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


@dataclass
class RunResult:
    labels: torch.Tensor      # int32 [H][W]
    centers: torch.Tensor     # float32 [K'][5]
    endpoints: torch.Tensor   # int32 [K'][2]
    counts: torch.Tensor      # int32 [K']


class Scalp:
    """One image size and superpixel count, with its own device workspace."""

    def __init__(self, width: int, height: int, k: int, device: str | torch.device = "cuda",
                 **params):
        self.grid: Grid = make_grid(width, height, k)
        self.params: Params = default_params(**params)
        self.device = torch.device(device)
        self.ws_bytes = L.workspace_bytes(self.grid)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    # shapes
    @property
    def H(self) -> int:
        return self.grid.height

    @property
    def W(self) -> int:
        return self.grid.width

    @property
    def K(self) -> int:
        return self.grid.num_sp

    def _params(self, **over) -> Params:
        return L.apply_overrides(Params.from_buffer_copy(self.params), over)

    def _img(self, lab, contour):
        _need(lab, (self.H, self.W, 3), torch.float32, "lab")
        if contour is not None:   # None: the library computes the prior (CONTOUR_GRADIENT)
            _need(contour, (self.H, self.W), torch.float32, "contour")

    def _ws(self):
        return _p(self.workspace), ctypes.c_size_t(self.ws_bytes)

    def new_state(self):
        dev = self.device
        return (torch.empty((self.K, 5), dtype=torch.float32, device=dev),
                torch.empty((self.K, 2), dtype=torch.int32, device=dev),
                torch.empty((self.H, self.W), dtype=torch.int32, device=dev),
                torch.empty((self.K,), dtype=torch.int32, device=dev))

    def prepare(self, lab, contour, stream=None) -> None:
        self._img(lab, contour)
        p = self._params()
        check(L.lib().scalp_prepare(ctypes.byref(self.grid), ctypes.byref(p), _p(lab),
                                    _p(contour), *self._ws(), _s(stream)), "scalp_prepare")

    def init_grid(self, lab=None, contour=None, stream=None, reuse_prepared=False, out=None):
        if not reuse_prepared:
            self._img(lab, contour)
        if out is None:
            centers, endpoints, labels, _ = self.new_state()
        else:
            centers, endpoints, labels = out
        p = self._params(reuse_prepared=int(reuse_prepared))
        check(L.lib().scalp_init_grid(ctypes.byref(self.grid), ctypes.byref(p), _p(lab),
                                      _p(contour), _p(centers), _p(endpoints), _p(labels),
                                      *self._ws(), _s(stream)), "scalp_init_grid")
        return centers, endpoints, labels

    def assign(self, lab, contour, centers, endpoints, labels=None, stream=None,
               reuse_prepared=False, **over) -> torch.Tensor:
        if not reuse_prepared:
            self._img(lab, contour)
        _need(centers, (self.K, 5), torch.float32, "centers")
        _need(endpoints, (self.K, 2), torch.int32, "endpoints")
        if labels is None:
            labels = torch.empty((self.H, self.W), dtype=torch.int32, device=self.device)
        _need(labels, (self.H, self.W), torch.int32, "labels")
        p = self._params(reuse_prepared=int(reuse_prepared), **over)
        check(L.lib().scalp_assign(ctypes.byref(self.grid), ctypes.byref(p), _p(lab),
                                   _p(contour), _p(centers), _p(endpoints), _p(labels),
                                   *self._ws(), _s(stream)), "scalp_assign")
        return labels

    def update(self, lab, labels, centers, endpoints, stream=None, **over):
        """Returns new (centers, endpoints, counts); the inputs are not modified."""
        _need(lab, (self.H, self.W, 3), torch.float32, "lab")
        _need(labels, (self.H, self.W), torch.int32, "labels")
        _need(centers, (self.K, 5), torch.float32, "centers")
        _need(endpoints, (self.K, 2), torch.int32, "endpoints")
        c = centers.clone()
        e = endpoints.clone()
        counts = torch.empty((self.K,), dtype=torch.int32, device=self.device)
        p = self._params(**over)
        check(L.lib().scalp_update(ctypes.byref(self.grid), ctypes.byref(p), _p(lab), _p(labels),
                                   _p(c), _p(e), _p(counts), *self._ws(), _s(stream)),
              "scalp_update")
        return c, e, counts

    def assign_accumulate(self, centers, endpoints, labels, stream=None, **over) -> None:
        """One fused assignment pass on the packed image in the workspace; the
        update's sums stay in the workspace until finalize()."""
        p = self._params(**over)
        check(L.lib().scalp_assign_accumulate(ctypes.byref(self.grid), ctypes.byref(p),
                                              _p(centers), _p(endpoints), _p(labels),
                                              *self._ws(), _s(stream)),
              "scalp_assign_accumulate")

    def finalize(self, labels, centers, endpoints, counts, stream=None, **over) -> None:
        """Update (in place) from the sums left by assign_accumulate()."""
        p = self._params(**over)
        check(L.lib().scalp_finalize(ctypes.byref(self.grid), ctypes.byref(p), _p(labels),
                                     _p(centers), _p(endpoints), _p(counts), *self._ws(),
                                     _s(stream)), "scalp_finalize")

    def run(self, lab, contour, stream=None, out=None, **over) -> RunResult:
        self._img(lab, contour)
        centers, endpoints, labels, counts = out if out is not None else self.new_state()
        p = self._params(**over)
        check(L.lib().scalp_run(ctypes.byref(self.grid), ctypes.byref(p), _p(lab), _p(contour),
                                _p(centers), _p(endpoints), _p(labels), _p(counts),
                                *self._ws(), _s(stream)), "scalp_run")
        return RunResult(labels, centers, endpoints, counts)

    def run_static(self, lab, contour, stream=None, out=None, **over) -> RunResult:
        """run() through scalp_run_static: the library's device scratch instead of
        a workspace.  The call itself allocates nothing when `out` holds the
        four output tensors (new_state())."""
        self._img(lab, contour)
        centers, endpoints, labels, counts = out if out is not None else self.new_state()
        p = self._params(**over)
        check(L.lib().scalp_run_static(ctypes.byref(self.grid), ctypes.byref(p), _p(lab),
                                       _p(contour), _p(centers), _p(endpoints), _p(labels),
                                       _p(counts), _s(stream)), "scalp_run_static")
        return RunResult(labels, centers, endpoints, counts)

    def graph(self, centers, endpoints, labels, counts, **over) -> "Graph":
        """hipGraph of the iteration loop on these buffers (the packed image must
        already be in the workspace)."""
        p = self._params(**over)
        h = ctypes.c_void_p()
        check(L.lib().scalp_graph_create(ctypes.byref(self.grid), ctypes.byref(p), _p(centers),
                                         _p(endpoints), _p(labels), _p(counts), *self._ws(),
                                         ctypes.byref(h)), "scalp_graph_create")
        return Graph(h, keep=(self, centers, endpoints, labels, counts))


class Graph:
    def __init__(self, handle: ctypes.c_void_p, keep=()):
        self.handle = handle
        self._keep = keep

    def launch(self, stream=None) -> None:
        check(L.lib().scalp_graph_launch(self.handle, _s(stream)), "scalp_graph_launch")

    def close(self) -> None:
        if self.handle:
            check(L.lib().scalp_graph_destroy(self.handle), "scalp_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


class ScalpBatch:
    """A ragged batch: images of different sizes and superpixel counts,
    concatenated pixel-wise, run by one persistent launch per iteration."""

    def __init__(self, shapes: list[tuple[int, int, int]], device="cuda", **params):
        self.grids = [make_grid(w, h, k) for (w, h, k) in shapes]
        descs = []
        pix = sp = 0
        for g in self.grids:
            d = BatchDesc()
            d.pix_offset = pix
            d.sp_offset = sp
            d.grid = g
            descs.append(d)
            pix += g.width * g.height
            sp += g.num_sp
        self.descs = (BatchDesc * len(descs))(*descs)
        self.n = len(descs)
        self.total_pixels = pix
        self.total_sp = sp
        self.params = default_params(**params)
        self.device = torch.device(device)
        self.ws_bytes = int(L.lib().scalp_batch_workspace_bytes(self.descs, self.n))
        if self.ws_bytes == 0:
            raise ValueError("invalid batch")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def pixel_slices(self):
        out = []
        for d in self.descs:
            n = d.grid.width * d.grid.height
            out.append((d.pix_offset, d.pix_offset + n, d.grid.height, d.grid.width))
        return out

    def sp_slices(self):
        return [(d.sp_offset, d.sp_offset + d.grid.num_sp) for d in self.descs]

    def new_state(self):
        dev = self.device
        return (torch.empty((self.total_sp, 5), dtype=torch.float32, device=dev),
                torch.empty((self.total_sp, 2), dtype=torch.int32, device=dev),
                torch.empty((self.total_pixels,), dtype=torch.int32, device=dev),
                torch.empty((self.total_sp,), dtype=torch.int32, device=dev))

    def _check(self, lab, contour):
        _need(lab, (self.total_pixels, 3), torch.float32, "lab")
        if contour is not None:   # None: the library computes the prior (CONTOUR_GRADIENT)
            _need(contour, (self.total_pixels,), torch.float32, "contour")

    def run(self, lab, contour, stream=None, out=None, **over):
        self._check(lab, contour)
        centers, endpoints, labels, counts = out if out is not None else self.new_state()
        p = L.apply_overrides(Params.from_buffer_copy(self.params), over)
        check(L.lib().scalp_run_batched(self.descs, self.n, ctypes.byref(p), _p(lab), _p(contour),
                                        _p(centers), _p(endpoints), _p(labels), _p(counts),
                                        _p(self.workspace), ctypes.c_size_t(self.ws_bytes),
                                        _s(stream)), "scalp_run_batched")
        return centers, endpoints, labels, counts

    def graph(self, lab, contour, centers, endpoints, labels, counts, **over) -> Graph:
        self._check(lab, contour)
        p = L.apply_overrides(Params.from_buffer_copy(self.params), over)
        h = ctypes.c_void_p()
        check(L.lib().scalp_batched_graph_create(self.descs, self.n, ctypes.byref(p), _p(lab),
                                                 _p(contour), _p(centers), _p(endpoints),
                                                 _p(labels), _p(counts), _p(self.workspace),
                                                 ctypes.c_size_t(self.ws_bytes), ctypes.byref(h)),
              "scalp_batched_graph_create")
        return Graph(h, keep=(self, lab, contour, centers, endpoints, labels, counts))
