"""Soft (differentiable) SCALP: torch wrappers and autograd.Function.

The forward and the hand-written backward both run in libscalp.so
(scalp_soft_forward / scalp_soft_backward); path samples are recomputed in
the backward pass, never stored.  Layouts: lab [B][H][W][3], contour
[B][H][W], Q [B][9][H][W] (slot j = (di+1)*3 + (dj+1) of the 3x3 cell
neighbourhood), centres [B][K'][5] = (l, a, b, x, y).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from ._lib import Params, check, default_params, make_grid
from .scalp import _need, _p, _s


class SoftScalp:
    """Soft SCALP for batches of `batch` images of one size."""

    def __init__(self, width: int, height: int, k: int, batch: int, temperature: float = 0.5,
                 device="cuda", **params):
        params.setdefault("iterations", 5)
        self.grid = make_grid(width, height, k)
        self.params: Params = default_params(**params)
        self.T = float(temperature)
        self.B = int(batch)
        self.device = torch.device(device)
        g = ctypes.byref(self.grid)
        self.saved_bytes = int(L.lib().scalp_soft_saved_bytes(g, self.B, self.params.iterations))
        self.ws_bytes = int(L.lib().scalp_soft_workspace_bytes(g, self.B))
        if self.saved_bytes == 0 or self.ws_bytes == 0:
            raise ValueError("invalid soft SCALP configuration")
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    @property
    def K(self) -> int:
        return self.grid.num_sp

    @property
    def iterations(self) -> int:
        return self.params.iterations

    def _check(self, lab, contour):
        H, W = self.grid.height, self.grid.width
        _need(lab, (self.B, H, W, 3), torch.float32, "lab")
        _need(contour, (self.B, H, W), torch.float32, "contour")

    def forward(self, lab, contour, stream=None):
        """Returns (centres_t [T+1][B][K'][5], q_t [T][B][9][H][W], saved bytes)."""
        self._check(lab, contour)
        H, W, T = self.grid.height, self.grid.width, self.iterations
        dev = self.device
        centers_t = torch.empty((T + 1, self.B, self.K, 5), dtype=torch.float32, device=dev)
        q_t = torch.empty((T, self.B, 9, H, W), dtype=torch.float32, device=dev)
        saved = torch.empty(self.saved_bytes, dtype=torch.uint8, device=dev)
        check(L.lib().scalp_soft_forward(ctypes.byref(self.grid), ctypes.byref(self.params),
                                         ctypes.c_float(self.T), self.B, _p(lab), _p(contour),
                                         _p(centers_t), _p(q_t), _p(saved), _p(self.workspace),
                                         ctypes.c_size_t(self.ws_bytes), _s(stream)),
              "scalp_soft_forward")
        return centers_t, q_t, saved

    def backward(self, lab, contour, centers_t, q_t, saved, grad_q, grad_centers, stream=None):
        """dL/dlab, dL/dcontour given dL/dQ_T [B][9][H][W] and dL/dTheta_T [B][K'][5]."""
        self._check(lab, contour)
        H, W = self.grid.height, self.grid.width
        _need(grad_q, (self.B, 9, H, W), torch.float32, "grad_q")
        _need(grad_centers, (self.B, self.K, 5), torch.float32, "grad_centers")
        glab = torch.empty_like(lab)
        gcon = torch.empty_like(contour)
        check(L.lib().scalp_soft_backward(ctypes.byref(self.grid), ctypes.byref(self.params),
                                          ctypes.c_float(self.T), self.B, _p(lab), _p(contour),
                                          _p(centers_t), _p(q_t), _p(saved), _p(grad_q),
                                          _p(grad_centers), _p(glab), _p(gcon),
                                          _p(self.workspace), ctypes.c_size_t(self.ws_bytes),
                                          _s(stream)), "scalp_soft_backward")
        return glab, gcon


class ScalpSoftFunction(torch.autograd.Function):
    """(lab, contour) -> (Q_T [B][9][H][W], Theta_T [B][K'][5])."""

    @staticmethod
    def forward(ctx, lab, contour, engine: SoftScalp):
        lab = lab.contiguous()
        contour = contour.contiguous()
        centers_t, q_t, saved = engine.forward(lab, contour)
        ctx.engine = engine
        ctx.save_for_backward(lab, contour, centers_t, q_t, saved)
        return q_t[-1], centers_t[-1]

    @staticmethod
    def backward(ctx, grad_q, grad_theta):
        lab, contour, centers_t, q_t, saved = ctx.saved_tensors
        eng = ctx.engine
        if grad_q is None:
            grad_q = torch.zeros_like(q_t[-1])
        if grad_theta is None:
            grad_theta = torch.zeros_like(centers_t[-1])
        glab, gcon = eng.backward(lab, contour, centers_t, q_t, saved,
                                  grad_q.contiguous().float(), grad_theta.contiguous().float())
        return glab, gcon, None


def scalp_soft(lab: torch.Tensor, contour: torch.Tensor, engine: SoftScalp):
    """Differentiable soft SCALP: returns (Q_T, Theta_T)."""
    return ScalpSoftFunction.apply(lab, contour, engine)
