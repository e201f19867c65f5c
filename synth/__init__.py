"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This package holds no arithmetic of the smoothing method: it only
draws images and parameter sets."""
from .voronoi import voronoi_image, batch_mix, FrameSpec, train_crop_specs  # noqa: F401
from .degraded import clipart_image, hdr_image, texture_image  # noqa: F401
