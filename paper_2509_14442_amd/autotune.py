"""Autotuner for the launch shape and checkpoint stride of a batch of scenes.

It times the forward (and, for mode "fwd+adj", render and adjoint) of the given scenes
with HIP events on the current stream for a list of candidates, and caches the winner
as JSON keyed by (gfx arch, storage dtype, tracer, samples per pixel, step-cap bucket,
grid-size bucket, ray-count bucket, scene count, mode). A key missing from the user's
cache is looked up in the table shipped with the package (autotune_table.json, winners
this same tuner measured on an MI355X), and only then tuned. On return the scenes carry
the chosen checkpoint stride; the entry's "source" says where it came from ("cache",
"table" or "measured").
Run it before capturing a graph: tuning launches kernels and allocates buffers.
"""

from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import api

DEFAULT_CACHE = os.environ.get("RBOS_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "rbos", "autotune.json"))
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_table.json")

# (tile, waves per block, persistent, blocks per CU; 0 = each kernel's occupancy limit)
LAUNCHES: List[Tuple[Tuple[int, int], int, bool, int]] = [
    ((8, 8), 4, False, 0),
    ((8, 8), 2, False, 0),
    ((8, 8), 1, False, 0),
    ((16, 4), 4, False, 0),
    ((32, 2), 4, False, 0),
    ((64, 1), 4, False, 0),
    ((8, 8), 4, True, 0),
    ((8, 8), 2, True, 0),
    ((8, 8), 4, True, 2),
]
# 1: every step stored (24 B per ray-step), no replay; 3, 4: chunks that record their
# samples for the reverse; 6: chunks of 6 at 4 wavefronts per SIMD; 8, 16, 32, 64: chunks
# of 8
STRIDES = (1, 3, 4, 6, 8, 16, 32, 64)
LAYOUTS = ("cell", "xpair")


def _bucket(x: float) -> int:
    return int(round(math.log2(max(x, 1.0))))


def cache_key(scenes: Sequence[api.Scene], mode: str) -> str:
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(dev, "gcnArchName", "gfx").split(":")[0]
    vox = sum(s.dims[0] * s.dims[1] * s.dims[2] for s in scenes) / max(len(scenes), 1)
    rays = sum(s.n_rays for s in scenes)
    dtype = scenes[0].field.dtype if scenes else "f32"
    tracer = int(scenes[0].struct.tracer) if scenes else 0
    spp = max((s.spp for s in scenes), default=1)
    steps = max((int(s.struct.max_steps) for s in scenes), default=1)
    return (f"v4|{arch}|{dtype}|t{tracer}|spp{spp}|m{_bucket(steps)}|g{_bucket(vox)}|r{_bucket(rays)}"
            f"|n{len(scenes)}|{mode}")


def ckpt_bytes(scenes: Sequence[api.Scene], stride: int) -> int:
    """Checkpoint bytes of the scenes at this stride (as the library sizes them)."""
    import ctypes as C

    tot = 0
    for s in scenes:
        st = C.c_int32(s.struct.ckpt_stride)
        s.struct.ckpt_stride = stride
        tot += api.lib().rbos_ckpt_bytes(C.byref(s.struct))
        s.struct.ckpt_stride = st.value
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


def _warm(fn, seconds: float) -> None:
    """Run fn back to back for about `seconds`, so that the first candidates are not timed
    while the device clocks are still rising."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        fn()
        torch.cuda.synchronize()


def _entry_of(launch_t) -> Dict:
    (tw, th), wpb, pers, bpc = launch_t
    return {"tile": [tw, th], "waves_per_block": wpb, "persistent": bool(pers), "blocks_per_cu": bpc}


def tune(scenes: List[api.Scene], mode: str = "fwd+adj", targets: Optional[List[torch.Tensor]] = None,
         strides: Sequence[int] = STRIDES, launches=LAUNCHES, layouts: Sequence[str] = LAYOUTS,
         hbm_budget: Optional[int] = None, reps: int = 3, cache: Optional[str] = DEFAULT_CACHE,
         force: bool = False, table: Optional[str] = TABLE) -> Dict:
    """Pick launch shapes, the checkpoint stride and the field layout for these scenes;
    returns the cached or new entry {"fwd": launch, "adj": launch, "ckpt_stride", "layout",
    "ms"} (a launch is {"tile", "waves_per_block", "persistent", "blocks_per_cu"}; "adj" is
    absent for mode "fwd"). The scenes come back with the chosen stride; the layout is the
    caller's to apply (Field.relayout).

    After a short warm-up, stage 1 times the forward trace (with checkpoints at stride 16
    unless mode is "fwd") for every launch shape, stage 2 the adjoint alone for every shape
    after one forward with the best forward shape, stage 3 the whole forward + render + adjoint for every
    stride whose checkpoints fit `hbm_budget` (default: half the free device memory), then the
    adjoint alone again for every shape at the chosen stride (the adjoint's form depends on
    the stride), stage 4 the best of those with the scenes' fields re-encoded in each other
    layout. With force
    the cache and the table are not consulted."""
    key = cache_key(scenes, mode)
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            db = json.load(f)
    if not force:
        entry, source = db.get(key), "cache"
        if entry is None and table and os.path.exists(table):
            with open(table) as f:
                entry, source = json.load(f).get(key), "table"
        if entry is not None:
            for s in scenes:
                s.struct.ckpt_stride = entry["ckpt_stride"]
            return dict(entry, source=source)
    if hbm_budget is None:
        free, _ = torch.cuda.mem_get_info()
        hbm_budget = int(free * 0.5)
    if targets is None:
        targets = [None] * len(scenes)
    tg = [t if t is not None else torch.zeros(s.n_pixels, device="cuda") for t, s in zip(targets, scenes)]
    adj = mode != "fwd"

    def tracer(fwd_t, adj_t, stride):
        for s in scenes:
            s.struct.ckpt_stride = stride
        return api.Tracer(scenes, api.make_launch(*fwd_t), checkpoints=adj,
                          adjoint_launch=api.make_launch(*adj_t) if adj_t is not None else None)

    default_stride = 16 if adj else 0
    _warm(tracer(launches[0], None, default_stride).forward, 0.3)
    fwd_ms = [(_time(tracer(lt, None, default_stride).forward, reps), lt) for lt in launches]
    fwd_ms.sort(key=lambda x: x[0])
    best_fwd = fwd_ms[0][1]
    entry = {"fwd": _entry_of(best_fwd), "ckpt_stride": default_stride, "ms": fwd_ms[0][0]}
    if adj:
        grads = [torch.zeros(tuple(reversed(s.dims)), dtype=torch.float64, device="cuda") for s in scenes]
        adj_ms = []
        for lt in launches:
            tr = tracer(best_fwd, lt, default_stride)
            tr.forward()
            tr.render(tg)
            adj_ms.append((_time(lambda: tr.adjoint(grads, zero=False), reps), lt))
            del tr
        adj_ms.sort(key=lambda x: x[0])
        best_adj = adj_ms[0][1]

        def whole(stride):
            tr = tracer(best_fwd, best_adj, stride)

            def step():
                tr.forward()
                tr.render(tg)
                tr.adjoint(grads, zero=False)

            return _time(step, reps)

        best = (whole(default_stride), default_stride)
        for st in strides:
            if st == default_stride or ckpt_bytes(scenes, st) > hbm_budget:
                continue
            ms = whole(st)
            if ms < best[0]:
                best = (ms, st)
        if best[1] != default_stride:
            # the adjoint's form follows the stride, and so does its best launch
            first_adj, adj_ms = best_adj, []
            for lt in launches:
                tr = tracer(best_fwd, lt, best[1])
                tr.forward()
                tr.render(tg)
                adj_ms.append((_time(lambda: tr.adjoint(grads, zero=False), reps), lt))
                del tr
            adj_ms.sort(key=lambda x: x[0])
            if adj_ms[0][1] != first_adj:
                best_adj = adj_ms[0][1]
                ms = whole(best[1])
                if ms < best[0]:
                    best = (ms, best[1])
                else:
                    best_adj = first_adj
        entry.update({"adj": _entry_of(best_adj), "ckpt_stride": best[1], "ms": best[0]})
    own = scenes[0].field.layout if scenes else "cell"
    entry["layout"] = own
    for lay in layouts:
        if lay == own or not scenes:
            continue
        fields = [s.field for s in scenes]
        try:
            for s in scenes:
                s.set_field(s.field.relayout(lay))
            if adj:
                ms = whole(entry["ckpt_stride"])
            else:
                ms = _time(tracer(best_fwd, None, 0).forward, reps)
        finally:
            for s, f in zip(scenes, fields):
                s.set_field(f)
        if ms < entry["ms"]:
            entry.update({"layout": lay, "ms": ms})
    for s in scenes:
        s.struct.ckpt_stride = entry["ckpt_stride"]
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        db[key] = entry
        with open(cache, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
    return dict(entry, source="measured")


def launch_of(entry: Dict, which: str = "fwd"):
    """The tuned launch of the forward ("fwd") or adjoint ("adj") kernel."""
    e = entry[which]
    return api.make_launch(tuple(e["tile"]), e["waves_per_block"], e["persistent"], e["blocks_per_cu"])
