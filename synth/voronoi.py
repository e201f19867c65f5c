"""Seeded Voronoi + Gaussian-detail images.

Stand-in for the natural photographs the paper times and shows (QVGA to 4K,
grey and colour); none of those images is available, so every workload here
is synthetic:

* centres: K points uniform in [0, H) x [0, W) (drawn first);
* each pixel (y, x) takes the nearest centre by plain (non-periodic)
  Euclidean distance (scipy cKDTree; ties are a measure-zero event);
* intensities: C x K uniform in [0, 1) (drawn second), channels independent,
  geometry shared;
* detail: i.i.d. N(0, sigma^2) per pixel and channel (drawn third), added,
  clipped to [0, 1] and rounded to float32.

All draws come from numpy.random.default_rng(seed) (PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.spatial import cKDTree


def voronoi_image(H: int, W: int, C: int = 1, K: int = 40, sigma: float = 0.05,
                  seed: int = 0) -> np.ndarray:
    """float32 array (C, H, W) in [0, 1]."""
    rng = np.random.default_rng(seed)
    centres = rng.random((K, 2)) * np.array([H, W], dtype=np.float64)
    inten = rng.random((C, K))
    tree = cKDTree(centres)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64),
                         np.arange(W, dtype=np.float64), indexing="ij")
    _, label = tree.query(np.stack([yy.ravel(), xx.ravel()], axis=1), workers=-1)
    label = label.reshape(H, W)
    img = inten[:, label]
    img = img + sigma * rng.standard_normal((C, H, W))
    np.clip(img, 0.0, 1.0, out=img)
    return np.ascontiguousarray(img, dtype=np.float32)


@dataclass(frozen=True)
class FrameSpec:
    H: int
    W: int
    C: int
    lam: float
    p: float
    eps: float
    N: int
    seed: int
    K: int
    sigma: float

    def image(self) -> np.ndarray:
        return voronoi_image(self.H, self.W, self.C, self.K, self.sigma, self.seed)


# Cell density for the mixed batch follows the 1080p workload: 400 cells on
# 1920 x 1080, scaled with the pixel count (at least 40 cells).
_MIX_SIZES = [(480, 640), (720, 1280), (1080, 1920), (2160, 3840)]


def batch_mix(n: int = 64, seed: int = 2, first_image_seed: int = 1000,
              sizes=None) -> list[FrameSpec]:
    """Seeded mix of frame sizes (uniform over `sizes`), grey or RGB (uniform),
    lam ~ U[0.5, 2], p ~ U[0.5, 1], eps = 1e-4, N = 4; image i has seed
    first_image_seed + i."""
    sizes = _MIX_SIZES if sizes is None else sizes
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        H, W = sizes[int(rng.integers(len(sizes)))]
        C = (1, 3)[int(rng.integers(2))]
        lam = float(rng.uniform(0.5, 2.0))
        p = float(rng.uniform(0.5, 1.0))
        K = max(40, int(round(400 * H * W / (1920 * 1080))))
        out.append(FrameSpec(H, W, C, lam, p, 1e-4, 4, first_image_seed + i, K, 0.05))
    return out


def train_crop_specs(n: int, first_seed: int = 100000, H: int = 256, W: int = 256,
                     param_seed: int | None = None) -> list[FrameSpec]:
    """RGB crops for the learned surrogate: K ~ U{10..40} cells per crop,
    sigma = 0.05, lam ~ U[0.5, 2], p ~ U[0.5, 1], N = 4; crop i has image
    seed first_seed + i and its own parameter draws (seeded by the same)."""
    out = []
    for i in range(n):
        rng = np.random.default_rng((first_seed + i) if param_seed is None else param_seed + i)
        K = int(rng.integers(10, 41))
        lam = float(rng.uniform(0.5, 2.0))
        p = float(rng.uniform(0.5, 1.0))
        out.append(FrameSpec(H, W, 3, lam, p, 1e-4, 4, first_seed + i, K, 0.05))
    return out
