"""Seeded temperature fields on voxel centres.

Voxels are cell-centred: voxel i on an axis of n voxels over [lo, hi] sits at
lo + (i + 1/2) (hi - lo) / n. Fields are returned as float64 arrays indexed
[nz][ny][nx] (x fastest). Plumes are hot Gaussians,
T += A exp(-|x - x_c|^2 / (2 sigma^2)).
"""

from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

T_AMBIENT = 293.0  # K


@dataclasses.dataclass(frozen=True)
class Plume:
    centre: Tuple[float, float, float]
    amplitude: float  # K
    sigma: float  # m (standard deviation)


@dataclasses.dataclass(frozen=True)
class FieldSpec:
    plumes: Tuple[Plume, ...]
    strat_per_m: float = 0.0  # vertical stratification dT/dz, z = 0 at the floor
    t0: float = T_AMBIENT


def plume_unit_box(seed: int = 1) -> FieldSpec:
    """One 5 K plume, sigma 0.15 m, centre ~ U[0.3, 0.7]^3 (unit box)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, size=3)
    return FieldSpec((Plume(tuple(float(x) for x in c), 5.0, 0.15),), 0.0)


def plumes_room(seed: int = None, lo=(0.0, 0.0, 0.0), hi=(4.0, 4.0, 3.0), rng=None,
                n_range=(4, 8), amp_range=(1.0, 8.0), sigma_range=(0.1, 0.5),
                strat_per_m: float = 0.5) -> FieldSpec:
    """K ~ U{4..8} plumes. Per plume, in this draw order: sigma ~ U[0.1, 0.5] m,
    A ~ U[1, 8] K, then the centre uniform over the box shrunk on each axis by
    max(2 sigma, 0.1 extent). Plus 0.5 K/m stratification (warmer above)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    k = int(rng.integers(n_range[0], n_range[1] + 1))
    plumes: List[Plume] = []
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    ext = hi - lo
    for _ in range(k):
        sigma = float(rng.uniform(*sigma_range))
        amp = float(rng.uniform(*amp_range))
        margin = np.maximum(2.0 * sigma, 0.1 * ext)
        c = rng.uniform(lo + margin, hi - margin)
        plumes.append(Plume(tuple(float(x) for x in c), amp, sigma))
    return FieldSpec(tuple(plumes), strat_per_m)


def voxel_centres(lo: Sequence[float], hi: Sequence[float], dims: Sequence[int]):
    """Coordinates of voxel centres per axis: (xs, ys, zs)."""
    return tuple(
        lo[a] + (np.arange(dims[a], dtype=np.float64) + 0.5) * ((hi[a] - lo[a]) / dims[a])
        for a in range(3)
    )


def temperature_grid(spec: FieldSpec, lo, hi, dims) -> np.ndarray:
    """T on voxel centres, float64 [nz][ny][nx]."""
    xs, ys, zs = voxel_centres(lo, hi, dims)
    z3 = zs[:, None, None]
    y3 = ys[None, :, None]
    x3 = xs[None, None, :]
    T = np.full((dims[2], dims[1], dims[0]), spec.t0, dtype=np.float64)
    if spec.strat_per_m:
        T += spec.strat_per_m * (z3 - lo[2])
    for p in spec.plumes:
        cx, cy, cz = p.centre
        # separable evaluation: exp(-(dx^2+dy^2+dz^2)/(2 s^2))
        s2 = 2.0 * p.sigma * p.sigma
        ex = np.exp(-((x3 - cx) ** 2) / s2)
        ey = np.exp(-((y3 - cy) ** 2) / s2)
        ez = np.exp(-((z3 - cz) ** 2) / s2)
        T += p.amplitude * (ez * ey * ex)
    return T
