"""Shared test fixtures: seeded workloads prepared for the GPU path and for the oracle.

Both sides receive the same input arrays (temperature, pattern, pixel ids, targets);
the oracle computes its own eta - 1 and storage codes from them.
"""

from __future__ import annotations

import dataclasses
import os
import sys
from typing import Optional

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bos_inputs as bi  # noqa: E402
import oracle  # noqa: E402

RHO0G, T0 = 2.7e-4, 293.0
CODES = {"f32": oracle.CODE_F32, "f16": oracle.CODE_F16, "bf16": oracle.CODE_BF16}
# the x-pair storage formats hold the same codes as the cell records of their code type
CODES.update({k + "-xpair": v for k, v in list(CODES.items())})


@dataclasses.dataclass
class Workload:
    scene: bi.Scene
    T32: np.ndarray               # float32 [nz][ny][nx]
    pattern: np.ndarray           # float64 [pat_h][pat_w] (stored as float32 on both sides)
    pixel_ids: Optional[np.ndarray] = None

    @property
    def pattern32(self) -> np.ndarray:
        return self.pattern.astype(np.float32)


def unit_box_workload(width=64, height=64) -> Workload:
    sc = bi.scene_unit_box().replace(width=width, height=height)
    T = bi.temperature_grid(bi.plume_unit_box(1), sc.box_lo, sc.box_hi, sc.dims).astype(np.float32)
    return Workload(sc, T, bi.binary_dots(11))


def room_workload(dims=(128, 128, 128), width=512, height=512, seed=2, max_steps=512, ckpt=16,
                  pat=1024) -> Workload:
    sc = bi.scene_room(dims, width, height, max_steps, ckpt, pat=pat)
    T = bi.temperature_grid(bi.plumes_room(seed, sc.box_lo, sc.box_hi), sc.box_lo, sc.box_hi, sc.dims)
    return Workload(sc, T.astype(np.float32), bi.blurred_noise(12, (pat, pat)))


def expected_scale(T32: np.ndarray, dtype: str, offset: float = 0.0) -> float:
    """The power-of-two code scale for a temperature field, derived here from the seeded
    input: the largest s with s * max |eta - 1 - c| <= 2^14 (1 for FP32)."""
    if dtype.split("-")[0] == "f32":
        return 1.0
    t = T32.astype(np.float64)
    bound = max(abs(RHO0G * T0 / t.min() - offset), abs(RHO0G * T0 / t.max() - offset))
    return float(2.0 ** np.floor(np.log2(2.0 ** 14 / bound)))


def stored_delta(T32: np.ndarray, dtype: str = "f32", scale: float = 1.0, offset: float = 0.0) -> np.ndarray:
    """eta - 1 exactly as stored (the oracle's own binary32 arithmetic and codes), FP64."""
    d32 = oracle.delta_from_temperature_f32(T32, RHO0G, T0)
    codes = oracle.encode(d32, CODES[dtype], scale, offset)
    return oracle.decode(codes, CODES[dtype], scale, offset)


def oracle_scene(w: Workload):
    """Oracle view of the scene: the pattern as the float32 values both sides store."""
    return w.scene, w.pattern32.astype(np.float64)


def oracle_forward(w: Workload, delta: np.ndarray):
    F = oracle.grid_field(delta, w.scene.box_lo, w.scene.box_hi)
    out = oracle.trace(F, w.scene, w.pixel_ids)
    img, dI, st = oracle.render(w.scene, w.pattern32.astype(np.float64), out["uv"], out["status"])
    out.update(image=img, dI=dI, status_r=st)
    return F, out


def exit_error(uv_gpu: np.ndarray, uv_ref: np.ndarray) -> np.ndarray:
    """Euclidean distance in the wall plane (m)."""
    return np.sqrt(((uv_gpu.astype(np.float64) - uv_ref) ** 2).sum(axis=1))


def grad_errors(g: np.ndarray, ref: np.ndarray):
    """(L2-relative error, fraction of voxels outside the per-voxel bound)."""
    l2 = float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300))
    bound = 1e-3 * np.maximum(np.abs(ref), 1e-2 * np.abs(ref).max())
    frac = float(np.mean(np.abs(g - ref) > bound))
    return l2, frac


def bench_tuned(scenes):
    """The launch shapes and checkpoint stride bench.py times for these scenes (api.Scene
    objects, built as bench.py builds them): the autotuner's entry in the table shipped
    with the package, never a tuning run here. The scenes come back with its stride."""
    from paper_2509_14442_amd import autotune

    e = autotune.tune(scenes, "fwd+adj", cache=None)
    assert e["source"] == "table", e
    assert e["layout"] == "cell", e
    return autotune.launch_of(e), autotune.launch_of(e, "adj"), e["ckpt_stride"]

