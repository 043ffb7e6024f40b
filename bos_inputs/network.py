"""Seeded inputs of the network-field workloads: MLP parameters (a random initialisation
stands in for trained weights, which the paper does not publish), boundary points on the
inlet plane and collocation points in the box. Random numbers only: the layer layout is
the packed order of the parameter vector (per layer the weights [in][out] row-major, then
the biases), nothing of the network's evaluation."""

from __future__ import annotations

import numpy as np

N_OUT = 5


def mlp_param_shapes(width: int, depth: int):
    dims = [3] + [width] * depth + [N_OUT]
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def mlp_params(width: int, depth: int, seed: int, out_scale: float = 1.0, bias_std: float = 0.0) -> np.ndarray:
    """Glorot-uniform weights (the last layer scaled by out_scale) and biases drawn from
    N(0, bias_std^2), packed."""
    rng = np.random.default_rng(seed)
    shapes = mlp_param_shapes(width, depth)
    parts = []
    for i, (fi, fo) in enumerate(shapes):
        lim = np.sqrt(6.0 / (fi + fo))
        W = rng.uniform(-lim, lim, (fi, fo)) * (out_scale if i == len(shapes) - 1 else 1.0)
        b = rng.normal(0.0, bias_std, fo) if bias_std > 0 else np.zeros(fo)
        parts += [W.ravel(), b]
    return np.concatenate(parts)


def inlet_points(n: int, lo, hi, seed: int) -> np.ndarray:
    """n points uniform on the x = lo face (the inlet plane of the boundary loss)."""
    rng = np.random.default_rng(seed)
    return np.column_stack([np.full(n, lo[0]), rng.uniform(lo[1], hi[1], n), rng.uniform(lo[2], hi[2], n)])


def collocation_points(n: int, lo, hi, seed: int) -> np.ndarray:
    """n points uniform in the box (collocation points of the PDE loss)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (n, 3))
