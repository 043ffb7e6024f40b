"""Wall patterns: printed random binary dots and a blurred-noise projector image.

Both are float64 arrays [rows][cols], row 0 at the top. They stand in for the
paper's wavelet-noise projector pattern (Sec. 3.A), which is not available.
"""

from __future__ import annotations

import numpy as np


def binary_dots(seed: int = 11, size=(256, 256), fill: float = 0.3) -> np.ndarray:
    """Bernoulli(fill) texels in {0, 1}."""
    rng = np.random.default_rng(seed)
    return (rng.random(size) < fill).astype(np.float64)


def blurred_noise(seed: int = 12, size=(1024, 1024), sigma_px: float = 1.0) -> np.ndarray:
    """U[0,1) greyscale, Gaussian-blurred with sigma 1 px (reflect boundary, 4 sigma)."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    img = rng.random(size)
    return gaussian_filter(img, sigma=sigma_px, mode="reflect", truncate=4.0)
