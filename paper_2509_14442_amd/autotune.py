"""Autotuner for the launch shape and checkpoint stride of a batch of scenes.

It times the forward (and, for mode "fwd+adj", render and adjoint) of the given scenes
with HIP events on the current stream for a list of candidates, and caches the winner
as JSON keyed by (gfx arch, storage dtype, grid-size bucket, ray-count bucket, mode).
Run it before capturing a graph: tuning launches kernels and allocates buffers.
"""

from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import api

DEFAULT_CACHE = os.environ.get("RBOS_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "rbos", "autotune.json"))

# (tile, waves per block, persistent, blocks per CU)
LAUNCHES: List[Tuple[Tuple[int, int], int, bool, int]] = [
    ((8, 8), 4, False, 8),
    ((8, 8), 2, False, 8),
    ((16, 4), 4, False, 8),
    ((8, 8), 4, True, 3),
    ((8, 8), 4, True, 6),
]
STRIDES = (8, 16, 32)


def _bucket(x: float) -> int:
    return int(round(math.log2(max(x, 1.0))))


def cache_key(scenes: Sequence[api.Scene], mode: str) -> str:
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(dev, "gcnArchName", "gfx").split(":")[0]
    vox = sum(s.dims[0] * s.dims[1] * s.dims[2] for s in scenes) / max(len(scenes), 1)
    rays = sum(s.n_rays for s in scenes)
    dtype = scenes[0].field.dtype if scenes else "f32"
    return f"{arch}|{dtype}|g{_bucket(vox)}|r{_bucket(rays)}|n{len(scenes)}|{mode}"


def ckpt_bytes(scenes: Sequence[api.Scene], stride: int) -> int:
    tot = 0
    for s in scenes:
        slots = (s.desc.max_steps - 1) // stride
        tot += (19 + 6 * slots) * s.n_rays * 4
    return tot


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(scenes: List[api.Scene], mode: str = "fwd+adj", targets: Optional[List[torch.Tensor]] = None,
         strides: Sequence[int] = STRIDES, launches=LAUNCHES, hbm_budget: Optional[int] = None,
         reps: int = 2, cache: Optional[str] = DEFAULT_CACHE, force: bool = False) -> Dict:
    """Pick (launch, checkpoint stride) for these scenes; returns the cached or new entry
    {"tile", "waves_per_block", "persistent", "blocks_per_cu", "ckpt_stride", "ms"}."""
    key = cache_key(scenes, mode)
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
        if key in db and not force:
            return db[key]
    if hbm_budget is None:
        free, _ = torch.cuda.mem_get_info()
        hbm_budget = int(free * 0.5)
    if targets is None:
        targets = [None] * len(scenes)
    best = None

    def run_cfg(launch_t, stride):
        launch = api.make_launch(*launch_t)
        for s in scenes:
            s.struct.ckpt_stride = stride
        tr = api.Tracer(scenes, launch, checkpoints=(mode != "fwd"))
        if mode == "fwd":
            return _time(lambda: tr.forward(), reps)
        tg = [t if t is not None else torch.zeros(s.n_rays, device="cuda") for t, s in zip(targets, scenes)]
        grads = [torch.zeros(tuple(reversed(s.dims)), dtype=torch.float64, device="cuda") for s in scenes]

        def step():
            tr.forward()
            tr.render(tg)
            tr.adjoint(grads, zero=False)

        return _time(step, reps)

    # stage 1: launch shape at the default stride; stage 2: stride with the best shape
    default_stride = 16 if mode != "fwd" else 0
    results = []
    for lt in launches:
        ms = run_cfg(lt, default_stride)
        results.append((ms, lt, default_stride))
    results.sort(key=lambda x: x[0])
    best_lt = results[0][1]
    best = results[0]
    if mode != "fwd":
        for st in strides:
            if st == default_stride or ckpt_bytes(scenes, st) > hbm_budget:
                continue
            ms = run_cfg(best_lt, st)
            if ms < best[0]:
                best = (ms, best_lt, st)
    for s in scenes:
        s.struct.ckpt_stride = best[2]
    (tw, th), wpb, pers, bpc = best[1]
    entry = {"tile": [tw, th], "waves_per_block": wpb, "persistent": bool(pers), "blocks_per_cu": bpc,
             "ckpt_stride": best[2], "ms": best[0]}
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        db[key] = entry
        with open(cache, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return entry


def launch_of(entry: Dict):
    return api.make_launch(tuple(entry["tile"]), entry["waves_per_block"], entry["persistent"],
                           entry["blocks_per_cu"])
