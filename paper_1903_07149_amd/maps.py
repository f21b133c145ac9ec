"""Per-pixel maps through libscalp.so (argument marshalling only): the
multi-scale boundary map and the on-device contour prior, plus the
multi-scale decomposition of one image in a single batched run."""
from __future__ import annotations

import ctypes
import torch

from . import _lib as L
from .scalp import ScalpBatch, _p, _s


def boundary_map(labels: torch.Tensor, stream=None) -> torch.Tensor:
    """labels: int32 [n][H][W] on the GPU -> float32 [H][W] boundary frequency."""
    if labels.dtype != torch.int32 or labels.dim() != 3:
        raise TypeError("labels must be int32 [n][H][W]")
    labels = labels.contiguous()
    n, H, W = labels.shape
    out = torch.empty((H, W), dtype=torch.float32, device=labels.device)
    L.check(L.lib().scalp_boundary_map(W, H, _p(labels), n, _p(out), _s(stream)),
            "scalp_boundary_map")
    return out


def contour_from_lab(lab: torch.Tensor, stream=None) -> torch.Tensor:
    """lab: float32 [H][W][3] on the GPU -> contour prior float32 [H][W] in [0, 1]."""
    if lab.dtype != torch.float32 or lab.dim() != 3 or lab.shape[2] != 3:
        raise TypeError("lab must be float32 [H][W][3]")
    lab = lab.contiguous()
    H, W, _ = lab.shape
    out = torch.empty((H, W), dtype=torch.float32, device=lab.device)
    ws = torch.empty(4096, dtype=torch.uint8, device=lab.device)
    L.check(L.lib().scalp_contour_from_lab(W, H, _p(lab), _p(out), _p(ws), ctypes.c_size_t(4096),
                                           _s(stream)), "scalp_contour_from_lab")
    return out


def scales(n: int = 12, kmin: int = 6, kmax: int = 600) -> list[int]:
    """n superpixel counts from kmin to kmax, evenly spaced in log k."""
    return [int(round(kmin * (kmax / kmin) ** (i / (n - 1)))) for i in range(n)]


class MultiScale:
    """Decompositions of one image at several k, run as one ragged batch (one
    persistent launch per iteration), and their boundary-frequency map."""

    def __init__(self, width: int, height: int, ks: list[int] | None = None, **params):
        self.ks = ks or scales()
        self.W, self.H = width, height
        self.batch = ScalpBatch([(width, height, k) for k in self.ks], **params)

    def stack(self, lab: torch.Tensor, contour: torch.Tensor | None):
        """The image (and its contour map, if given) repeated once per scale,
        in the batch's concatenated layout."""
        return self.stack_of(len(self.ks), lab, contour)

    @staticmethod
    def stack_of(n: int, lab: torch.Tensor, contour: torch.Tensor | None):
        """The image (and its contour map, if given) repeated n times."""
        lab_b = lab.reshape(1, -1, 3).expand(n, -1, -1).reshape(-1, 3).contiguous()
        con_b = None if contour is None else contour.reshape(1, -1).expand(n, -1).reshape(-1).contiguous()
        return lab_b, con_b

    def run(self, lab: torch.Tensor, contour: torch.Tensor | None, stream=None):
        """lab float32 [H][W][3], contour float32 [H][W] (None with
        contour_source=CONTOUR_GRADIENT) -> (labels int32 [n][H][W], boundary
        frequency float32 [H][W])."""
        lab_b, con_b = self.stack(lab, contour)
        c, e, l, cnt = self.batch.run(lab_b, con_b, stream=stream)
        labels = l.reshape(len(self.ks), self.H, self.W)
        return labels, boundary_map(labels, stream=stream)
