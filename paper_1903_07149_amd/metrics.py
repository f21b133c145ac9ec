"""Superpixel quality metrics of Sec. III-A.2 (BR, ASA, UE, CO) through
libscalp.so's `scalp_metrics` (argument marshalling only)."""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .scalp import _p, _s


def metrics(labels: torch.Tensor, gt: torch.Tensor, num_sp: int | None = None,
            num_regions: int | None = None, epsilon: float = 2.0, stream=None) -> dict:
    """labels, gt: int32 [H][W] GPU tensors.  Returns {br, asa, ue, co,
    gt_boundary, sp_boundary}."""
    if labels.dtype != torch.int32 or gt.dtype != torch.int32:
        raise TypeError("labels and gt must be int32")
    if labels.shape != gt.shape or labels.dim() != 2:
        raise ValueError("labels and gt must be [H][W] of the same shape")
    labels = labels.contiguous()
    gt = gt.contiguous()
    H, W = labels.shape
    K = int(num_sp if num_sp is not None else int(labels.max().item()) + 1)
    R = int(num_regions if num_regions is not None else int(gt.max().item()) + 1)
    nb = int(L.lib().scalp_metrics_workspace_bytes(W, H, K, R))
    if nb == 0:
        raise ValueError("metric table too large or sizes invalid")
    ws = torch.empty(nb, dtype=torch.uint8, device=labels.device)
    out = torch.empty(6, dtype=torch.float64, device=labels.device)
    L.check(L.lib().scalp_metrics(W, H, _p(labels), K, _p(gt), R, ctypes.c_float(epsilon), _p(out),
                                  _p(ws), ctypes.c_size_t(nb), _s(stream)), "scalp_metrics")
    v = out.cpu().tolist()
    return {"br": v[0], "asa": v[1], "ue": v[2], "co": v[3], "gt_boundary": int(v[4]),
            "sp_boundary": int(v[5])}


class Metrics:
    """Reusable `scalp_metrics` call for one shape: workspace and result are
    allocated once; `run` only enqueues (no host synchronisation) and
    returns the device result double[6] = {BR, ASA, UE, CO, number of
    ground-truth boundary pixels, number of superpixel boundary pixels}."""

    def __init__(self, width: int, height: int, num_sp: int, num_regions: int,
                 epsilon: float = 2.0, device="cuda"):
        self.W, self.H, self.K, self.R = int(width), int(height), int(num_sp), int(num_regions)
        self.epsilon = float(epsilon)
        self.nb = int(L.lib().scalp_metrics_workspace_bytes(self.W, self.H, self.K, self.R))
        if self.nb == 0:
            raise ValueError("metric table too large or sizes invalid")
        self.ws = torch.empty(self.nb, dtype=torch.uint8, device=device)
        self.out = torch.empty(6, dtype=torch.float64, device=device)

    def run(self, labels: torch.Tensor, gt: torch.Tensor, stream=None) -> torch.Tensor:
        if labels.dtype != torch.int32 or gt.dtype != torch.int32:
            raise TypeError("labels and gt must be int32")
        if tuple(labels.shape) != (self.H, self.W) or tuple(gt.shape) != (self.H, self.W):
            raise ValueError("labels and gt must be [H][W] of the configured shape")
        if not (labels.is_contiguous() and gt.is_contiguous()):
            raise ValueError("labels and gt must be contiguous")
        L.check(L.lib().scalp_metrics(self.W, self.H, _p(labels), self.K, _p(gt), self.R,
                                      ctypes.c_float(self.epsilon), _p(self.out), _p(self.ws),
                                      ctypes.c_size_t(self.nb), _s(stream)), "scalp_metrics")
        return self.out
