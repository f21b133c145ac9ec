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
