"""Seeded synthetic inputs for the SCALP clustering path.

The paper evaluates on natural photographs with a learned soft contour map
(Sec. III-A.1 and Sec. II-E).  Neither the images nor the detector are
available, so every workload here is synthetic: a Voronoi partition of the
image plane, one random sRGB colour per region (optionally with a smooth
linear colour ramp inside the region), i.i.d. Gaussian noise, quantisation
to 8 bits, conversion to CIELab (the feature space of Sec. II-A), and a soft
contour prior in [0, 1] (the map C of Sec. II-D) taken as the normalised
gradient magnitude of the noise-free image.

This module holds no arithmetic of the clustering method itself: it only
produces inputs.  Both the CPU oracle tests and the GPU path draw from it.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.spatial import cKDTree

# sRGB (IEC 61966-2-1) primaries to CIE XYZ, D65 white.
_RGB_TO_XYZ = np.array(
    [[0.4124, 0.3576, 0.1805],
     [0.2126, 0.7152, 0.0722],
     [0.0193, 0.1192, 0.9505]], dtype=np.float64)
_WHITE_D65 = np.array([0.95047, 1.0, 1.08883], dtype=np.float64)


def _srgb_to_linear(c: np.ndarray) -> np.ndarray:
    c = np.asarray(c, dtype=np.float64) / 255.0
    return np.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)


_LIN_LUT = _srgb_to_linear(np.arange(256))


def _lab_f(t: np.ndarray) -> np.ndarray:
    d = 6.0 / 29.0
    return np.where(t > d ** 3, np.cbrt(t), t / (3.0 * d * d) + 4.0 / 29.0)


def rgb_to_lab(rgb: np.ndarray) -> np.ndarray:
    """sRGB in [0, 255] (uint8 or float) -> CIELab, float64, shape (..., 3)."""
    if rgb.dtype == np.uint8:
        lin = _LIN_LUT[rgb]
    else:
        lin = _srgb_to_linear(np.clip(rgb, 0.0, 255.0))
    xyz = lin @ _RGB_TO_XYZ.T
    f = _lab_f(xyz / _WHITE_D65)
    lab = np.empty_like(f)
    lab[..., 0] = 116.0 * f[..., 1] - 16.0
    lab[..., 1] = 500.0 * (f[..., 0] - f[..., 1])
    lab[..., 2] = 200.0 * (f[..., 1] - f[..., 2])
    return lab


def gradient_contour(lab_clean: np.ndarray) -> np.ndarray:
    """Normalised central-difference gradient magnitude (replicated borders)."""
    p = np.pad(lab_clean, ((1, 1), (1, 1), (0, 0)), mode="edge")
    gx = 0.5 * (p[1:-1, 2:, :] - p[1:-1, :-2, :])
    gy = 0.5 * (p[2:, 1:-1, :] - p[:-2, 1:-1, :])
    mag = np.sqrt(np.sum(gx * gx + gy * gy, axis=2))
    mx = float(mag.max()) if mag.size else 0.0
    if mx > 0.0:
        mag = mag / mx
    else:
        mag = np.zeros_like(mag)
    return mag.astype(np.float32)


@dataclasses.dataclass
class Image:
    lab: np.ndarray      # float32 [H][W][3]
    contour: np.ndarray  # float32 [H][W], values in [0, 1]
    gt: np.ndarray       # int32 [H][W], Voronoi region id (synthetic ground truth)

    @property
    def height(self) -> int:
        return self.lab.shape[0]

    @property
    def width(self) -> int:
        return self.lab.shape[1]


def make_image(width: int, height: int, regions: int, noise_sigma: float,
               seed: int | np.random.Generator, ramps: bool = False) -> Image:
    """One synthetic Voronoi image (see the module docstring for the recipe)."""
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    W, H, R = int(width), int(height), int(regions)
    sx = rng.uniform(0.0, W, R)
    sy = rng.uniform(0.0, H, R)
    yy, xx = np.mgrid[0:H, 0:W]
    pts = np.stack([xx.ravel(), yy.ravel()], axis=1).astype(np.float64)
    _, gt = cKDTree(np.stack([sx, sy], axis=1)).query(pts, k=1, workers=-1)
    gt = gt.reshape(H, W).astype(np.int32)
    colours = rng.integers(0, 256, (R, 3)).astype(np.float64)
    clean = colours[gt]                               # float64 [H][W][3]
    if ramps:
        d = np.sqrt(W * H / R)
        grad = rng.normal(0.0, 20.0 / d, (R, 3, 2))
        rel = np.stack([xx - sx[gt], yy - sy[gt]], axis=-1)   # [H][W][2]
        clean = clean + np.einsum("hwcj,hwj->hwc", grad[gt], rel)
        clean = np.clip(clean, 0.0, 255.0)
    noisy = clean + rng.normal(0.0, noise_sigma, clean.shape)
    rgb8 = np.clip(np.rint(noisy), 0, 255).astype(np.uint8)
    lab = rgb_to_lab(rgb8).astype(np.float32)
    contour = gradient_contour(rgb_to_lab(clean if ramps else clean.astype(np.uint8)))
    return Image(lab=np.ascontiguousarray(lab), contour=contour, gt=gt)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    width: int
    height: int
    regions: int
    noise_sigma: float
    seed: int
    k: int
    iterations: int
    ramps: bool = False


# The five workloads of the build, with the shapes and statistics of the
# paper's setting (Sec. III-A: 321x481 images, 5 iterations) scaled up.
BSD_SHAPE = Workload("voronoi_481x321_k250", 481, 321, 40, 10.0, 1, 250, 10)
HD = Workload("voronoi_1920x1080_k2000", 1920, 1080, 400, 8.0, 2, 2000, 10, ramps=True)
UHD = Workload("voronoi_3840x2160_k10000", 3840, 2160, 1500, 8.0, 3, 10000, 10)

BATCH_IMAGES = 64
BATCH_SEED0 = 400
SOFT_BATCH = 16
SOFT_SEED0 = 500


def workload_image(w: Workload) -> Image:
    return make_image(w.width, w.height, w.regions, w.noise_sigma, w.seed, ramps=w.ramps)


def batch_workloads(n: int = BATCH_IMAGES, seed0: int = BATCH_SEED0,
                    lo: int = 240, hi: int = 2160, per_px: int = 1000) -> list[Workload]:
    """Ragged batch: H, W ~ U{lo..hi}, regions ~ U{20..800}, k = round(HW / per_px)."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        h = int(rng.integers(lo, hi + 1))
        w = int(rng.integers(lo, hi + 1))
        reg = int(rng.integers(20, 801))
        k = max(1, int(round(h * w / per_px)))
        out.append(Workload(f"batch{i}_{w}x{h}", w, h, reg, 10.0, seed0 + i, k, 10))
    return out


def soft_workloads(n: int = SOFT_BATCH, size: int = 512) -> list[Workload]:
    return [Workload(f"soft{b}_{size}x{size}", size, size, 100, 10.0, SOFT_SEED0 + b, 400, 5)
            for b in range(n)]


def random_lab(width: int, height: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Unstructured noise image (uniform Lab box) and a uniform [0,1] contour map,
    for small randomised tests."""
    rng = np.random.default_rng(seed)
    lab = np.empty((height, width, 3), np.float32)
    lab[..., 0] = rng.uniform(0.0, 100.0, (height, width))
    lab[..., 1:] = rng.uniform(-80.0, 80.0, (height, width, 2))
    contour = rng.uniform(0.0, 1.0, (height, width)).astype(np.float32)
    return lab, contour
