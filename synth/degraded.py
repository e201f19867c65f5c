"""Seeded stand-ins for the inputs of the Welsch-penalty workloads (clip-art
compression-artifact removal, texture smoothing).  The paper's images are not
available; these generators give images of the same kind:

* clipart_image: flat Voronoi cells (no detail noise) put through a block
  transform coder: each 8 x 8 block (edge-padded to a multiple of 8, then
  cropped back) is taken to the orthonormal 2-D DCT-II, every coefficient
  (u, v) is rounded to a multiple of q (1 + u + v), and the block is
  transformed back.  That leaves blocking and ringing around cell edges, the
  artifacts the paper removes.  Clipped to [0, 1], float32.
* texture_image: Voronoi cells, each carrying a sinusoidal stripe texture of
  its own orientation, period (4 .. 10 px) and phase, amplitude amp, plus
  N(0, sigma^2) detail.  Clipped to [0, 1], float32.

Draws come from numpy.random.default_rng(seed) in the order: centres,
intensities, then (texture only) orientations, periods, phases, noise.
"""
from __future__ import annotations

import numpy as np
from scipy.fft import dctn, idctn
from scipy.spatial import cKDTree


def _labels(rng, H, W, K):
    centres = rng.random((K, 2)) * np.array([H, W], dtype=np.float64)
    tree = cKDTree(centres)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    _, label = tree.query(np.stack([yy.ravel(), xx.ravel()], axis=1), workers=-1)
    return label.reshape(H, W), yy, xx


def clipart_image(H: int, W: int, C: int = 3, K: int = 60, q: float = 0.03, seed: int = 0) -> np.ndarray:
    """float32 (C, H, W): flat cells with 8 x 8 block-coding artifacts."""
    rng = np.random.default_rng(seed)
    label, _, _ = _labels(rng, H, W, K)
    inten = rng.random((C, K))
    img = inten[:, label]
    Hp, Wp = -(-H // 8) * 8, -(-W // 8) * 8
    img = np.pad(img, ((0, 0), (0, Hp - H), (0, Wp - W)), mode="edge")
    blocks = img.reshape(C, Hp // 8, 8, Wp // 8, 8)
    coef = dctn(blocks, type=2, axes=(2, 4), norm="ortho")
    u = np.arange(8)
    step = q * (1.0 + u[:, None] + u[None, :])  # step for coefficient (u, v)
    coef = np.round(coef / step[None, None, :, None, :]) * step[None, None, :, None, :]
    img = idctn(coef, type=2, axes=(2, 4), norm="ortho").reshape(C, Hp, Wp)[:, :H, :W]
    np.clip(img, 0.0, 1.0, out=img)
    return np.ascontiguousarray(img, dtype=np.float32)


def texture_image(H: int, W: int, C: int = 3, K: int = 30, amp: float = 0.2, sigma: float = 0.02,
                  seed: int = 0) -> np.ndarray:
    """float32 (C, H, W): cells carrying oriented stripe textures."""
    rng = np.random.default_rng(seed)
    label, yy, xx = _labels(rng, H, W, K)
    inten = rng.random((C, K))
    theta = rng.random(K) * np.pi
    period = 4.0 + 6.0 * rng.random(K)
    phase = rng.random(K) * 2.0 * np.pi
    t = theta[label]
    stripes = np.sin(2.0 * np.pi * (xx * np.cos(t) + yy * np.sin(t)) / period[label] + phase[label])
    img = inten[:, label] + amp * stripes[None] + sigma * rng.standard_normal((C, H, W))
    np.clip(img, 0.0, 1.0, out=img)
    return np.ascontiguousarray(img, dtype=np.float32)


def hdr_image(H: int, W: int, K: int = 60, decades: float = 4.0, sigma: float = 0.02, seed: int = 0) -> np.ndarray:
    """float32 (3, H, W) linear radiance spanning about `decades` orders of
    magnitude: 10 ** (decades * v) of a colour Voronoi image v (cells in
    [0, 1), N(0, sigma^2) detail, clipped to [0, 1]).  Stand-in for the HDR
    radiance maps the paper tone-maps."""
    from .voronoi import voronoi_image
    v = voronoi_image(H, W, 3, K, sigma, seed=seed).astype(np.float64)
    return np.ascontiguousarray(10.0 ** (decades * v), dtype=np.float32)
