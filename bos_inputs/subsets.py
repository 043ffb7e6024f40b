"""Seeded pixel subsets (pixel id j = row * width + col)."""

from __future__ import annotations

import numpy as np


def pixel_subset(n_pixels: int, count: int, seed: int = 15) -> np.ndarray:
    """`count` distinct pixel ids drawn without replacement, returned sorted (int32)."""
    rng = np.random.default_rng(seed)
    ids = rng.choice(n_pixels, size=min(count, n_pixels), replace=False)
    return np.sort(ids).astype(np.int32)


def strided_tiles(width: int, height: int, tile: int = 8, keep_every: int = 4,
                  offset: int = 0) -> np.ndarray:
    """Pixel ids of every `keep_every`-th tile x tile block (row-major over blocks):
    a coherent, evenly spread subset of a full image."""
    tw = (width + tile - 1) // tile
    th = (height + tile - 1) // tile
    ids = []
    for b in range(offset, tw * th, keep_every):
        by, bx = divmod(b, tw)
        rows = np.arange(by * tile, min(by * tile + tile, height))
        cols = np.arange(bx * tile, min(bx * tile + tile, width))
        ids.append((rows[:, None] * width + cols[None, :]).ravel())
    return np.concatenate(ids).astype(np.int32) if ids else np.zeros(0, np.int32)
