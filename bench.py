#!/usr/bin/env python3
"""Benchmark: BOS ray tracing forward and forward+adjoint on one MI355X.

Workload H: the 4 x 4 x 3 m room with a 128^3 voxel field (seeded hot plumes plus
0.5 K/m stratification), a 1024 x 1024 pinhole camera (1,048,576 rays), Sharma RK4 with
h = 0.5 voxel and at most 512 steps, checkpoints every 16 steps, projector pattern
1024 x 1024 (blurred uniform noise). Inputs are synthetic and seeded.

One timed step = the whole hot path on resident inputs: encode the field from
temperature, trace every ray with checkpoints, render + L_BOS + dL/d(u, v), zero the
FP64 gradient, adjoint. value = ray-steps / step time (ray-steps = sum of per-ray Sharma
steps inside the box, read back from the kernel output).

Prints one JSON line (rank 0). See the design doc for the roofline and algorithmic counts.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ray-steps/s fwd and fwd+adjoint (128^3 field, 1M rays) vs FP64 err; % HBM/L2"

# Algorithmic FP32 work per ray-step (flops, FMA = 2); derivation in the design doc.
FLOP_FWD_STEP = 200
FLOP_ADJ_STEP = 700
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32 (published)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    p.add_argument("--offset", type=float, default=0.0, help="16-bit code offset c (eta - 1 = c + q/s)")
    p.add_argument("--ckpt", type=int, default=16)
    p.add_argument("--tile", default="8x8")
    p.add_argument("--wpb", type=int, default=4)
    p.add_argument("--persistent", type=int, default=0)
    p.add_argument("--blocks-per-cu", type=int, default=8)
    p.add_argument("--graph", type=int, default=1, help="replay the step as a captured HIP graph")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time for the CPU baseline")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--traffic", default=None, help="JSON file with measured HBM bytes per adjoint launch")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1; sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import bos_inputs as bi
    from paper_2509_14442_amd import api

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    desc = bi.scene_h().replace(ckpt_stride=args.ckpt)
    lo, hi, dims = desc.box_lo, desc.box_hi, desc.dims
    TA = bi.temperature_grid(bi.plumes_room(3, lo, hi), lo, hi, dims).astype(np.float32)
    TB = bi.temperature_grid(bi.plumes_room(4, lo, hi), lo, hi, dims).astype(np.float32)
    pat_np = bi.blurred_noise(12, (desc.pat_h, desc.pat_w)).astype(np.float32)

    tA = torch.from_numpy(TA).to(dev)
    tB = torch.from_numpy(TB).to(dev)
    pat = torch.from_numpy(pat_np).to(dev)
    tw, th = (int(x) for x in args.tile.split("x"))
    launch = api.make_launch((tw, th), args.wpb, bool(args.persistent), args.blocks_per_cu)

    fieldA = api.Field.from_temperature(tA, args.dtype, None, args.offset)
    fieldB = api.Field.from_temperature(tB, args.dtype, fieldA.scale, args.offset)
    # measured image: the render of field B (outside the timed region)
    trB = api.Tracer([api.Scene(desc, fieldB, pat)], launch, checkpoints=False)
    trB.forward().render()
    target = trB.image[0].clone()

    scene = api.Scene(desc, fieldA, pat)
    tr = api.Tracer([scene], launch, checkpoints=True)
    grad = torch.zeros((dims[2], dims[1], dims[0]), dtype=torch.float64, device=dev)
    fwd_only = api.Tracer([scene], launch, checkpoints=False)

    def step():
        fieldA.encode_temperature(tA)
        tr.forward()
        tr.render([target])
        grad.zero_()
        tr.adjoint([grad], zero=False)

    # warm up (also allocates every buffer the step uses)
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    ray_steps = int(tr.n_steps[0].sum(dtype=torch.int64))
    loss = float(tr.loss[0])

    graph = None
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        g_eager = grad.clone()
        step()
        torch.cuda.synchronize()
        # every replay must reproduce the eager result
        assert torch.allclose(grad, g_eager, rtol=1e-9, atol=1e-12 * float(g_eager.abs().max())), \
            "graph replay differs from the eager step"

    # timed region: whole steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps

    # per-kernel timing with HIP events on the stream the kernels run on
    cur = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    acc = np.zeros(5)
    for _ in range(args.steps):
        ev[0].record(cur)
        fieldA.encode_temperature(tA)
        ev[1].record(cur)
        tr.forward()
        ev[2].record(cur)
        tr.render([target])
        ev[3].record(cur)
        grad.zero_()
        ev[4].record(cur)
        tr.adjoint([grad], zero=False)
        ev[5].record(cur)
        torch.cuda.synchronize()
        acc += [ev[i].elapsed_time(ev[i + 1]) for i in range(5)]
    k_ms = acc / args.steps
    # forward only (no checkpoints) + render
    evf = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd_ms = 0.0
    for _ in range(args.steps):
        evf[0].record(cur)
        fwd_only.forward()
        evf[1].record(cur)
        fwd_only.render([target])
        evf[2].record(cur)
        torch.cuda.synchronize()
        fwd_ms += evf[0].elapsed_time(evf[2])
    fwd_ms /= args.steps
    fwd_steps = int(fwd_only.n_steps[0].sum(dtype=torch.int64))
    assert fwd_steps == ray_steps

    adj_s = k_ms[4] * 1e-3
    achieved = FLOP_ADJ_STEP * ray_steps / adj_s / 1e12
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        with open(args.traffic) as f:
            traffic = json.load(f).get("adjoint_hbm_bytes_per_launch")
    out = {
        "metric": METRIC,
        "value": ray_steps / (ms_step * 1e-3),
        "unit": "ray-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": "H: 128^3 room field (4x4x3 m, seeded plumes + 0.5 K/m), 1024x1024 rays, "
                        "Sharma RK4 h=0.5 voxel, <=512 steps, checkpoint stride %d, projector 1024^2" % args.ckpt,
            "storage": args.dtype, "offset": args.offset, "tile": args.tile, "waves_per_block": args.wpb,
            "persistent": bool(args.persistent), "graph": bool(args.graph),
        },
        "ray_steps": ray_steps,
        "loss": loss,
        "fwd_ray_steps_per_s": ray_steps / (fwd_ms * 1e-3),
        "fwd_ms": fwd_ms,
        "kernel_ms": {"field_encode": k_ms[0], "trace_fwd_ckpt": k_ms[1], "render_loss": k_ms[2],
                      "grad_zero": k_ms[3], "trace_adjoint": k_ms[4]},
        "roofline": {
            "kernel": "k_trace_adj (adjoint)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic,
            "flop_per_ray_step": FLOP_ADJ_STEP,
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"], out["err"] = cpu_baseline_and_errors(args, desc, TA, TB, pat_np, tr, fieldA, pat,
                                                                 launch)
    print(json.dumps(out), flush=True)


def cpu_baseline_and_errors(args, desc, TA, TB, pat_np, tr, fieldA, pat, launch):
    """The FP64 oracle (test infrastructure) timed on a bounded, evenly spread sample of the
    same rays; the GPU's outputs on that sample are compared with it."""
    import numpy as np
    import torch

    import bos_inputs as bi
    import oracle
    from paper_2509_14442_amd import api

    oracle.build()
    p64 = pat_np.astype(np.float64)

    def stored(T):
        return oracle.decode(oracle.encode(oracle.delta_from_temperature_f32(T), oracle.CODE_F32),
                             oracle.CODE_F32)

    FA = oracle.grid_field(stored(TA), desc.box_lo, desc.box_hi)
    FB = oracle.grid_field(stored(TB), desc.box_lo, desc.box_hi)

    def run(ids):
        tb = oracle.trace(FB, desc, ids)
        target, _, _ = oracle.render(desc, p64, tb["uv"], tb["status"])
        t0 = time.perf_counter()
        fa = oracle.trace(FA, desc, ids)
        img, dI, st = oracle.render(desc, p64, fa["uv"], fa["status"])
        L, dL = oracle.loss(img, target, dI)
        g = oracle.adjoint(FA, desc, dL, ids)
        return time.perf_counter() - t0, fa, dL, g, target

    # calibrate on a small sample, then size the sample for ~cpu_seconds of oracle work
    probe = bi.strided_tiles(desc.width, desc.height, 8, 256, 7)
    dt, fa, _, _, _ = run(probe)
    per_ray = dt / max(len(probe), 1)
    n_target = int(args.cpu_seconds / max(per_ray, 1e-9))
    total_tiles = ((desc.width + 7) // 8) * ((desc.height + 7) // 8)
    keep = max(1, int(total_tiles * 64 / max(n_target, 1)))
    ids = bi.strided_tiles(desc.width, desc.height, 8, keep, 3)
    dt, fa, dL, g_ref, target = run(ids)
    steps = int(fa["n_steps"].sum())
    cpu = {"value": steps / dt, "unit": "ray-steps/s", "cores": oracle.threads(), "kind": "oracle",
           "sample": f"{len(ids)} rays (every {keep}th 8x8 tile of the 1024x1024 image), "
                     f"{steps} ray-steps, fwd+render+loss+adjoint in FP64, {dt:.1f} s"}

    # GPU vs oracle on the sample: exit points from the full timed run, gradient from the
    # adjoint restricted to the sample with the oracle's dL/d(u, v)
    uv = tr.uv[0].cpu().numpy().astype(np.float64)[ids]
    duv = tr.duv[0].cpu().numpy().astype(np.float64)[ids]
    ns = tr.n_steps[0].cpu().numpy()[ids]
    ok = np.isfinite(fa["uv"][:, 0])
    e_uv = np.sqrt(((uv[ok] - fa["uv"][ok]) ** 2).sum(1))
    e_duv = np.sqrt(((duv[ok] - fa["duv"][ok]) ** 2).sum(1))
    sub = api.Tracer([api.Scene(desc, fieldA, pat, torch.from_numpy(ids).cuda())], launch)
    sub.forward()
    lam = torch.from_numpy(dL.astype(np.float32)).cuda()
    g = sub.adjoint(dL_duv=[lam])[0].cpu().numpy()
    l2 = float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))
    bound = 1e-3 * np.maximum(np.abs(g_ref), 1e-2 * np.abs(g_ref).max())
    err = {
        "sample_rays": int(len(ids)),
        "exit_err_max_m": float(e_uv.max()), "exit_err_rms_m": float(np.sqrt((e_uv ** 2).mean())),
        "exit_err_p99_m": float(np.percentile(e_uv, 99)),
        "deflection_err_max_m": float(e_duv.max()),
        "bos_displacement_rms_m": float(np.sqrt((fa["duv"][ok] ** 2).sum(1).mean())),
        "n_steps_mismatch": int((ns != fa["n_steps"]).sum()),
        "grad_rel_l2": l2,
        "grad_voxel_fail_frac": float(np.mean(np.abs(g - g_ref) > bound)),
    }
    return cpu, err


if __name__ == "__main__":
    main()
