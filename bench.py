#!/usr/bin/env python3
"""Benchmark: BOS ray tracing forward and forward+adjoint on one MI355X.

Default workload (room1m): the 4 x 4 x 3 m room with a 128^3 voxel field (seeded hot plumes
plus 0.5 K/m stratification), a 1024 x 1024 pinhole camera (1,048,576 rays), Sharma RK4
with h = 0.5 voxel and at most 512 steps, projector pattern 1024 x 1024 (blurred uniform
noise). Inputs are synthetic and seeded. Launch shapes, checkpoint stride and field layout
come from the autotuner (its cache, else the table shipped with the package, else a tuning
run; --tune 2 forces one, --tune 0 takes the command line).

One timed step = the whole hot path on resident inputs, replayed as one captured HIP
graph: encode the field(s) from temperature, trace every ray with checkpoints, render +
L_BOS + dL/d(u, v), zero the FP64 gradient(s), adjoint. value = ray-steps / step time
(ray-steps = sum of per-ray Sharma steps inside the box, read back from the kernels).

Other workloads (--workload): batch64 = 64 scenes of uneven grids (48-192 per axis) and
cameras (128-1024 per side) in one persistent launch; room256 = 256 x 256 x 192 field,
2048 x 1536 rays, <= 1024 steps, with 16-bit storage (--dtype f16/bf16) and errors on a
4096-ray subsample.

Prints one JSON line.
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

# Algorithmic FP32 work per ray-step (flops, FMA = 2): one Sharma step (3 trilinear samples
# with gradient, 4 force flops each, stage arithmetic) ~200; its reverse with the replay of
# the step ~600 (the method's work, whatever an implementation recomputes).
FLOP_FWD_STEP = 200
FLOP_ADJ_STEP = 600
# Field values gathered per ray-step: 24 by the forward (3 samples of 8 corners), 48 by the
# adjoint (the replay's 24 and the reverse's 24), at 4 bytes (FP32) or 2 (16-bit codes).
GATHER_FWD_STEP = 24
GATHER_ADJ_STEP = 48
# Quasi-linear: 2 samples per step (a step's end point starts the next), and an adjoint
# without replay (2 samples with second derivatives and their reverse per step).
FLOP_FWD_STEP_QL = 150
FLOP_ADJ_STEP_QL = 320
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32 (published)
PEAK_HBM_BYTES_PER_S = 8.0e12  # MI355X HBM3E (published)
TRACERS = {"nonlinear": 0, "quasilinear": 1}


def parse(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="room1m", choices=["room1m", "batch64", "room256"])
    p.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"], help="code type of the stored field")
    p.add_argument("--layout", default="cell", choices=["cell", "xpair"],
                   help="field layout: cell records (8 corner codes per cell) or x-pairs (each voxel with its +x "
                        "neighbour)")
    p.add_argument("--tracer", default="nonlinear", choices=list(TRACERS),
                   help="nonlinear (Eq. 1 coupled) or quasi-linear (forces on the straight entry line)")
    p.add_argument("--offset", type=float, default=None,
                   help="16-bit code offset c (eta - 1 = c + q/s); default: the ambient eta - 1 (rho0G) for "
                        "16-bit storage, 0 for FP32. c = 0 with 16-bit storage misses the 1e-5 m exit bound")
    p.add_argument("--spp", type=int, default=1,
                   help="rays per pixel (Eq. 2 pixel integral over the triangular filter; 1 = pixel centres)")
    p.add_argument("--radiometry", type=int, default=0, choices=[0, 1],
                   help="weight each ray by |<n_w, v_w>| / |X_w - c|")
    p.add_argument("--sample-seed", type=int, default=1, help="sub-pixel sample key")
    p.add_argument("--field", default="grid", choices=["grid", "mlp"],
                   help="mlp: voxel temperatures from the network field, plus its boundary and PDE losses "
                        "(room1m only)")
    p.add_argument("--mlp-depth", type=int, default=4, help="network field: hidden layers of 64 units")
    p.add_argument("--pde-points", type=int, default=8192, help="network field: collocation points per step")
    p.add_argument("--boundary-points", type=int, default=4096, help="network field: inlet-plane points per step")
    p.add_argument("--ckpt", type=int, default=3,
                   help="checkpoint stride (steps) when not tuned: 3 and 4 record each chunk's samples for the "
                        "reverse, 6 replays chunks of 6, multiples of 8 chunks of 8, 1 stores every state")
    p.add_argument("--tile", default="8x8", help="forward: rays per wavefront tile")
    p.add_argument("--wpb", type=int, default=4, help="forward: wavefronts per block")
    p.add_argument("--persistent", type=int, default=0, help="forward: persistent blocks with tile queues")
    p.add_argument("--blocks-per-cu", type=int, default=0, help="persistent: 0 = the kernel's occupancy limit")
    p.add_argument("--adj-tile", default="8x8")
    p.add_argument("--adj-wpb", type=int, default=2)
    p.add_argument("--adj-persistent", type=int, default=1)
    p.add_argument("--adj-blocks-per-cu", type=int, default=0)
    p.add_argument("--graph", type=int, default=1, help="replay the step as a captured HIP graph")
    p.add_argument("--tune", type=int, default=1,
                   help="launch shapes, checkpoint stride and field layout from the autotuner: 1 its cache, "
                        "else the shipped table, else tune now; 2 tune now; 0 the command-line values")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time for the CPU baseline")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--counters", default=COUNTERS_FILE, help="summary of the counter runs of the tracer kernels")
    p.add_argument("--profile-kernels", action="store_true",
                   help="run the fixed dispatch sequence the counter runs profile (implies --tune 0) and exit")
    p.add_argument("--write-counters", default=None,
                   help="summarise the counter CSVs of --counter-dirs into this file (for the configuration the "
                        "other flags name) and exit")
    p.add_argument("--counter-dirs", nargs="*", default=[])
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run a plain device copy of known size (counter calibration) and exit")
    p.add_argument("--ceilings", action="store_true",
                   help="only measure the gather, FMA, FP64-atomic and HBM-copy ceilings and print them")
    p.add_argument("--no-ceilings", action="store_true", help="skip the live ceiling measurement")
    return p.parse_args(argv)


def storage(args) -> str:
    """Storage format of the field: the code type, with "-xpair" for the x-pair layout."""
    return args.dtype + ("-xpair" if args.layout == "xpair" else "")


def launches(args):
    """(forward launch, adjoint launch) given by the command line."""
    from paper_2509_14442_amd import api

    tw, th = (int(x) for x in args.tile.split("x"))
    fwd = api.make_launch((tw, th), args.wpb, bool(args.persistent), args.blocks_per_cu)
    tw, th = (int(x) for x in args.adj_tile.split("x"))
    adj = api.make_launch((tw, th), args.adj_wpb, bool(args.adj_persistent), args.adj_blocks_per_cu)
    return fwd, adj


# Hardware counters of the tracer kernels (rocprofv3 --pmc runs of `bench.py
# --profile-kernels`, summarised by `bench.py --write-counters`): vector-L1 accesses, L2
# requests and HBM bytes per launch. Used only while the kernels' sources hash to the value
# recorded with the counters and the configuration matches.
COUNTERS_FILE = os.path.join(ROOT, "profiles", "tracer_room1m_counters.md")
KERNEL_SOURCES = ("trace_fwd.hip", "trace_adj.hip", "rbos_device.hpp", "rbos_launch.hpp", "abi.hip",
                  "field_pack.hip", "ceilings.hip")
COPY_BYTES = 256 << 20
CEIL_COPY_BYTES = 1 << 30  # ceilings.measure's stream copy: bytes read (and written) per launch


def code_tokens(text: str) -> str:
    """C/C++ source without its comments, whitespace runs collapsed: edits to comments do
    not change what the counters were measured on."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":  # string or character literal, kept whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_14442_amd", "csrc", name), encoding="utf-8") as f:
            h.update(code_tokens(f.read()).encode())
    return h.hexdigest()


def launch_desc(l) -> dict:
    return {"tile": [int(l.tile_w), int(l.tile_h)], "waves_per_block": int(l.waves_per_block),
            "persistent": bool(l.persistent), "blocks_per_cu": int(l.blocks_per_cu)}


def _launch_str(l) -> str:
    return "%dx%d wpb %d persistent %d bpc %d" % (l.tile_w, l.tile_h, l.waves_per_block, l.persistent,
                                                  l.blocks_per_cu)


def counter_key(args, storage_name, ckpt, fwd_launch, adj_launch) -> str:
    """What the counters depend on: workload, tracer, storage, stride, samples and launches."""
    return ("%s|%s|%s|k%d|spp%d|radio%d|fwd %s|adj %s" % (args.workload, args.tracer, storage_name, ckpt,
                                                           args.spp, args.radiometry, _launch_str(fwd_launch),
                                                           _launch_str(adj_launch)))


def read_counters(path, key):
    """Per-launch counters {name: value} of the block recorded for `key`, or None when there is
    none or the kernels have changed since."""
    if not path or not os.path.exists(path):
        return None
    blocks, cur = [], {}
    with open(path) as f:
        for line in f:
            if line.strip() == "---":
                blocks.append(cur)
                cur = {}
            elif line.startswith("    ") and ": " in line:
                k, v = line.strip().split(": ", 1)
                cur[k] = v
    blocks.append(cur)
    h = kernel_source_hash()
    for b in blocks:
        if b.get("key") == key and b.get("source_sha256") == h:
            return {k: float(v) for k, v in b.items() if k not in ("key", "source_sha256")}
    return None


# dispatches of `bench.py --profile-kernels`, in order: the forward of the target image and
# 3 forwards without checkpoints; 3 steps (forward with checkpoints, render, adjoint); then
# the ceilings with 2 warm-up launches and 1 timed launch each (the scattered gather twice:
# the L2-resident footprint, then the 1 GiB one). The last launch of each group is used.
PROFILE_GROUPS = {
    "fwd": ("k_trace_fwd", 1, 4),
    "fwdck": ("k_trace_fwd", 4, 7),
    "adj": ("k_trace_adj", 0, 3),
    "copy": ("k_copy", 0, 3),
    "gather": ("k_gather_coherent<32>", 0, 3),
    "l2gather": ("k_gather_scattered<32>", 0, 3),
}
COUNTER_NAMES = {
    "TCP_TOTAL_CACHE_ACCESSES_sum": "tcp_accesses", "TCP_TCC_READ_REQ_sum": "tcp_tcc_read_req",
    "TCP_TCC_WRITE_REQ_sum": "tcp_tcc_write_req", "TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum": "tcp_tcc_atomic_req",
    "TCC_HIT_sum": "tcc_hit", "TCC_MISS_sum": "tcc_miss", "TCC_REQ_sum": "tcc_req", "TCC_EA0_RDREQ_sum": "tcc_ea_rdreq",
    "FETCH_SIZE": "fetch_kib", "WRITE_SIZE": "write_kib", "SQ_INSTS_VALU": "valu_insts",
    "SQ_INSTS_VMEM_RD": "vmem_rd_insts", "SQ_INSTS_LDS": "lds_insts", "SQ_WAVES": "waves",
    "SQ_WAIT_INST_ANY": "wait_inst_any", "SQ_WAVE_CYCLES": "wave_cycles", "SQ_INSTS_SALU": "salu_insts",
    "SQ_INSTS_VALU_FMA_F32": "valu_fma_f32", "GRBM_GUI_ACTIVE": "gui_active",
}


def write_counters(args):
    """Summarise rocprofv3 counter_collection.csv files of a --profile-kernels run into a
    block of the counters file (replacing the block of the same configuration)."""
    import csv
    import glob

    import torch  # noqa: F401  (struct types only; no device use)

    from paper_2509_14442_amd import api

    fwd, adj = launches(args)
    key = counter_key(args, storage(args), args.ckpt, fwd, adj)
    per = {}  # (group, counter) -> value of the group's last dispatch
    for d in args.counter_dirs:
        for fn in glob.glob(os.path.join(d, "*counter_collection.csv")):
            disp = {}
            with open(fn) as f:
                for r in csv.DictReader(f):
                    kname = r["Kernel_Name"].replace("(anonymous namespace)::", "")
                    k = (int(r["Dispatch_Id"]), kname, r["Counter_Name"])
                    disp[k] = disp.get(k, 0.0) + float(r["Counter_Value"])
            for g, (pat, lo, hi) in PROFILE_GROUPS.items():
                ids = sorted({i for (i, kn, _) in disp if pat in kn})
                if len(ids) < hi:
                    continue
                last = ids[hi - 1]
                for (i, kn, cn), v in disp.items():
                    if i == last and cn in COUNTER_NAMES:
                        per[(g, COUNTER_NAMES[cn])] = v
    fetch_scale = CEIL_COPY_BYTES / 1024 / per[("copy", "fetch_kib")] if ("copy", "fetch_kib") in per else None
    write_scale = CEIL_COPY_BYTES / 1024 / per[("copy", "write_kib")] if ("copy", "write_kib") in per else None
    lines = ["    key: " + key, "    source_sha256: " + kernel_source_hash()]
    if fetch_scale and write_scale:
        lines += ["    calib.fetch_scale: %.4f" % fetch_scale, "    calib.write_scale: %.4f" % write_scale]
    for (g, c), v in sorted(per.items()):
        lines.append("    %s.%s: %.6g" % (g, c, v))
        if c == "fetch_kib" and fetch_scale:
            lines.append("    %s.hbm_read_bytes: %.6g" % (g, v * 1024 * fetch_scale))
        if c == "write_kib" and write_scale:
            lines.append("    %s.hbm_write_bytes: %.6g" % (g, v * 1024 * write_scale))
    block = "\n".join(lines)
    out = args.write_counters
    text = open(out).read() if os.path.exists(out) else ""
    head, blocks = text, []
    if "\n    key: " in text:
        head = text[:text.index("\n    key: ") + 1]
        blocks = [b for b in text[len(head):].split("\n    ---\n")]
    blocks = [b.rstrip("\n") for b in blocks if b.strip() and ("key: " + key + "\n") not in b + "\n"]
    blocks.append(block)
    if not head:
        head = ("# Hardware counters per launch of the tracer kernels (see `bench.py --write-counters`)\n\n")
    with open(out, "w") as f:
        f.write(head + "\n    ---\n".join(blocks) + "\n")
    print("wrote block", key, "to", out)


def profile_kernels(args, dev):
    """A fixed dispatch sequence for the counter runs (see PROFILE_GROUPS)."""
    import torch

    from paper_2509_14442_amd import ceilings

    W = Workload(args, dev)
    for _ in range(3):
        W.fwd_only.forward()
    for _ in range(3):
        W.step()
    torch.cuda.synchronize()
    ceilings.measure(dev, reps=1)
    torch.cuda.synchronize()
    print(json.dumps({"profiled": counter_key(args, W.fields[0].dtype, W.ckpt_stride, W.launch, W.adj_launch)}),
          flush=True)


def calibrate_copy():
    """A plain streaming kernel of known size: y = -x over COPY_BYTES of float32 (reads and
    writes COPY_BYTES each), three launches."""
    import torch

    x = torch.ones(COPY_BYTES // 4, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_read_bytes": COPY_BYTES, "copy_write_bytes": COPY_BYTES, "launches": 3}), flush=True)


class Workload:
    """Fields, scenes, tracer, targets and gradients of one benchmark configuration."""

    def __init__(self, args, dev):
        import numpy as np
        import torch

        import bos_inputs as bi
        from paper_2509_14442_amd import api

        self.args = args
        launch, adj_launch = launches(args)
        self.temps, self.fields, self.scenes, self.descs = [], [], [], []
        if args.workload in ("room1m", "room256"):
            desc = (bi.scene_room_1m() if args.workload == "room1m" else bi.scene_room_256_3m()).replace(
                ckpt_stride=args.ckpt, tracer=TRACERS[args.tracer], spp=args.spp, seed=args.sample_seed,
                radiometry=args.radiometry)
            seed_a, seed_b = (3, 4) if args.workload == "room1m" else (5, 6)
            lo, hi, dims = desc.box_lo, desc.box_hi, desc.dims
            TA = bi.temperature_grid(bi.plumes_room(seed_a, lo, hi), lo, hi, dims).astype(np.float32)
            TB = bi.temperature_grid(bi.plumes_room(seed_b, lo, hi), lo, hi, dims).astype(np.float32)
            pat_np = bi.blurred_noise(12, (desc.pat_h, desc.pat_w)).astype(np.float32)
            self.pat_np, self.TA_np, self.TB_np = pat_np, TA, TB
            pat = torch.from_numpy(pat_np).to(dev)
            tA = torch.from_numpy(TA).to(dev)
            fA = api.Field.from_temperature(tA, storage(args), None, args.offset)
            fB = api.Field.from_temperature(torch.from_numpy(TB).to(dev), storage(args), fA.scale, args.offset)
            trB = api.Tracer([api.Scene(desc, fB, pat)], launch, checkpoints=False)
            trB.forward().render()
            self.targets = [trB.image[0].clone()]
            del trB, fB
            self.temps, self.fields, self.descs = [tA], [fA], [desc]
            self.scenes = [api.Scene(desc, fA, pat)]
            self.pat = pat
            self.data_note = "synthetic: seeded plume fields; target = render of a second seeded field"
            if args.tune:
                launch, adj_launch = self._tune(self.scenes, self.targets)
        else:  # batch64
            pat = torch.from_numpy(bi.blurred_noise(12, (1024, 1024)).astype(np.float32)).to(dev)
            self.pat = pat
            for sc, spec in bi.scenes_batch(64):
                sc = sc.replace(ckpt_stride=args.ckpt, tracer=TRACERS[args.tracer], spp=args.spp,
                                seed=args.sample_seed, radiometry=args.radiometry)
                T = torch.from_numpy(bi.temperature_grid(spec, sc.box_lo, sc.box_hi, sc.dims).astype(np.float32))
                T = T.to(dev)
                f = api.Field.from_temperature(T, storage(args), None, args.offset)
                self.temps.append(T)
                self.fields.append(f)
                self.descs.append(sc)
                self.scenes.append(api.Scene(sc, f, pat))
            self.targets = [torch.zeros(s.n_pixels, device=dev) for s in self.scenes]
            self.data_note = "synthetic: 64 seeded plume fields; target image = 0"
            if args.tune:
                # tuned on the whole batch: an 8-scene subset picked a launch 2 % slower on all 64
                launch, adj_launch = self._tune(self.scenes, self.targets)
        self.launch, self.adj_launch = launch, adj_launch
        self.ckpt_stride = int(self.scenes[0].struct.ckpt_stride)
        self.tracer = api.Tracer(self.scenes, launch, checkpoints=True, adjoint_launch=adj_launch)
        self.fwd_only = api.Tracer(self.scenes, launch, checkpoints=False)
        self.grads = [torch.zeros(tuple(reversed(s.dims)), dtype=torch.float64, device=dev) for s in self.scenes]
        self.mlp = None
        if args.field == "mlp":
            self._setup_mlp(args, dev)

    def _tune(self, scenes, targets):
        """Autotune these scenes (launch shapes, stride, layout) and apply the result to them;
        returns the forward and adjoint launches."""
        from paper_2509_14442_amd import autotune

        entry = autotune.tune(scenes, "fwd+adj", targets, reps=3, force=self.args.tune == 2)
        for i, s in enumerate(scenes):
            s.struct.ckpt_stride = entry["ckpt_stride"]
            if entry["layout"] != s.field.layout:
                s.set_field(s.field.relayout(entry["layout"]))
                self.fields[i] = s.field
        self.tuned = entry
        return autotune.launch_of(entry), autotune.launch_of(entry, "adj")

    def _setup_mlp(self, args, dev):
        """Network field (Sec. 2.D): the voxel temperatures come from an MLP; the target
        image is the render of a second network's field; the boundary targets are that
        network's outputs on the inlet plane; collocation points are uniform in the box."""
        import numpy as np
        import torch

        import bos_inputs as bi
        from paper_2509_14442_amd import api

        if args.workload != "room1m":
            raise SystemExit("--field mlp runs on the room1m workload")
        desc = self.descs[0]
        lo, hi, dims = desc.box_lo, desc.box_hi, desc.dims
        self.T0, self.T_in = 293.0, 303.0
        D = args.mlp_depth

        def net(seed):
            th = bi.mlp_params(64, D, seed, out_scale=0.3, bias_std=0.05).astype(np.float32)
            return api.MLP(torch.from_numpy(th).to(dev), 64, D, lo, hi)

        self.mlp = net(3)
        target_net = net(4)
        _, TB = target_net.forward(grid=dims, want_out=False, T0=self.T0, T_in=self.T_in)
        fB = api.Field.from_temperature(TB.reshape(tuple(reversed(dims))), storage(args), self.fields[0].scale,
                                        args.offset)
        trB = api.Tracer([api.Scene(desc, fB, self.pat)], self.launch, checkpoints=False)
        trB.forward().render()
        self.targets = [trB.image[0].clone()]
        del trB, fB
        self.pts_b = torch.from_numpy(bi.inlet_points(args.boundary_points, lo, hi, 5).astype(np.float32)).to(dev)
        self.tgt_b, _ = target_net.forward(self.pts_b)
        tb = self.tgt_b.double()
        un = float(tb[:, 2:5].norm(dim=1).max())
        self.norms_b = [float(tb[:, 0].abs().max()), float(tb[:, 1].abs().max()), un, un, un]
        self.pts_c = torch.from_numpy(bi.collocation_points(args.pde_points, lo, hi, 6).astype(np.float32)).to(dev)
        self.pde = dict(Re=100.0, Pe=70.0, Ri=0.5, L=1.0, gamma=(1.0, 1.0, 1.0))
        self.dparams = torch.zeros_like(self.mlp.params)
        self.T_grid = None
        self.data_note = ("synthetic: temperatures from a seeded MLP; target = render of a second seeded MLP's "
                          "field; boundary data = its outputs on the inlet plane")

    def mlp_forward(self):
        dims = self.descs[0].dims
        _, self.T_grid = self.mlp.forward(grid=dims, want_out=False, T0=self.T0, T_in=self.T_in)
        self.fields[0].encode_temperature(self.T_grid.reshape(tuple(reversed(dims))))

    def mlp_backward(self):
        """BOS chain, boundary loss and PDE loss, all added into dparams."""
        from paper_2509_14442_amd import api

        dims = self.descs[0].dims
        self.dparams.zero_()
        seed = api.MLP.bos_seed(self.T_grid, self.grads[0].reshape(-1), self.T0, self.T_in)
        self.mlp.backward(seed, grid=dims, dparams=self.dparams)
        out_b, _ = self.mlp.forward(self.pts_b)
        dL_b, self.loss_b = api.fit_seed(out_b, self.tgt_b, self.norms_b)
        self.mlp.backward(dL_b, self.pts_b, dparams=self.dparams)
        P = self.pde
        self.loss_pde, _, _ = self.mlp.pde_loss(self.pts_c, P["Re"], P["Pe"], P["Ri"], P["L"], P["gamma"],
                                                dparams=self.dparams)

    def encode(self):
        if self.mlp is not None:
            self.mlp_forward()
            return
        for f, T in zip(self.fields, self.temps):
            f.encode_temperature(T)

    def step(self):
        self.encode()
        self.tracer.forward()
        self.tracer.render(self.targets)
        for g in self.grads:
            g.zero_()
        self.tracer.adjoint(self.grads, zero=False)
        if self.mlp is not None:
            self.mlp_backward()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.write_counters:
        write_counters(args)
        return
    if args.ceilings:
        import torch

        from paper_2509_14442_amd import ceilings

        torch.cuda.set_device(0)
        print(json.dumps({"ceilings": ceilings.measure("cuda:0")}), flush=True)
        return

    import numpy as np
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile_kernels:
        args.tune = 0
        profile_kernels(args, dev)
        return
    W = Workload(args, dev)
    tr = W.tracer

    for _ in range(max(args.warmup, 1)):
        W.step()
    torch.cuda.synchronize()
    ray_steps = int(sum(int(n.sum(dtype=torch.int64)) for n in tr.n_steps))
    loss = float(sum(float(l) for l in tr.loss))

    graph = None
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            W.step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            W.step()
        torch.cuda.synchronize()
        W.step()
        torch.cuda.synchronize()
        g_eager = [g.clone() for g in W.grads]
        p_eager = W.dparams.clone() if W.mlp is not None else None
        for _ in range(2):  # every replay reproduces the eager step
            graph.replay()
            torch.cuda.synchronize()
            for g, ge in zip(W.grads, g_eager):
                assert torch.allclose(g, ge, rtol=1e-9, atol=1e-12 * float(ge.abs().max()) + 1e-300)
            if p_eager is not None:
                assert torch.allclose(W.dparams, p_eager, rtol=1e-5, atol=1e-6 * float(p_eager.abs().max()))

    # timed region: whole steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            W.step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps

    # per-kernel timing with HIP events on the stream the kernels run on
    cur = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    acc = np.zeros(6)
    for _ in range(args.steps):
        ev[0].record(cur)
        W.encode()
        ev[1].record(cur)
        tr.forward()
        ev[2].record(cur)
        tr.render(W.targets)
        ev[3].record(cur)
        for g in W.grads:
            g.zero_()
        ev[4].record(cur)
        tr.adjoint(W.grads, zero=False)
        ev[5].record(cur)
        if W.mlp is not None:
            W.mlp_backward()
        ev[6].record(cur)
        torch.cuda.synchronize()
        acc += [ev[i].elapsed_time(ev[i + 1]) for i in range(6)]
    k_ms = acc / args.steps
    mlp_info = mlp_timing(args, W, cur) if W.mlp is not None else None
    fwd_ms = 0.0
    fwd_kernel_ms = 0.0
    for _ in range(args.steps):
        ev[0].record(cur)
        W.fwd_only.forward()
        ev[1].record(cur)
        W.fwd_only.render(W.targets)
        ev[2].record(cur)
        torch.cuda.synchronize()
        fwd_kernel_ms += ev[0].elapsed_time(ev[1])
        fwd_ms += ev[0].elapsed_time(ev[2])
    fwd_ms /= args.steps
    fwd_kernel_ms /= args.steps
    assert int(sum(int(n.sum(dtype=torch.int64)) for n in W.fwd_only.n_steps)) == ray_steps

    adj_s = k_ms[4] * 1e-3
    ql = args.tracer == "quasilinear"
    flop_adj = FLOP_ADJ_STEP_QL if ql else FLOP_ADJ_STEP
    flop_fwd = FLOP_FWD_STEP_QL if ql else FLOP_FWD_STEP
    achieved = flop_adj * ray_steps / adj_s / 1e12
    cnt = read_counters(args.counters, counter_key(args, W.fields[0].dtype, W.ckpt_stride, W.launch, W.adj_launch))
    traffic = None
    if cnt is not None and "adj.hbm_read_bytes" in cnt and "adj.hbm_write_bytes" in cnt:
        traffic = cnt["adj.hbm_read_bytes"] + cnt["adj.hbm_write_bytes"]
    ceil = None
    if not args.no_ceilings:
        from paper_2509_14442_amd import ceilings

        ceil = ceilings.measure(dev)
    n_rays = sum(s.n_rays for s in W.scenes)
    names = {
        "room1m": "128^3 room field (4x4x3 m, seeded plumes + 0.5 K/m), 1024x1024 rays, Sharma RK4 h=0.5 voxel, "
             "<=512 steps, checkpoint stride %d, projector 1024^2" % W.ckpt_stride,
        "batch64": "64 room scenes, grids 48-192 per axis, cameras 128-1024 per side (%d rays), one persistent "
              "launch per kernel, hipGraph" % n_rays,
        "room256": "256x256x192 room field, 2048x1536 rays, <=1024 steps, checkpoint stride %d" % W.ckpt_stride,
    }
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
        "data": W.data_note,
        "config": {
            "workload": names[args.workload] + (", quasi-linear tracer" if args.tracer == "quasilinear" else "")
            + (", %d rays per pixel (triangular filter)" % args.spp if args.spp > 1 else "")
            + (", radiometric weight" if args.radiometry else ""),
            "tracer": args.tracer, "spp": args.spp, "radiometry": bool(args.radiometry),
            "storage": W.fields[0].dtype, "offset": W.fields[0].offset, "ckpt_stride": W.ckpt_stride,
            "fwd_launch": launch_desc(W.launch), "adj_launch": launch_desc(W.adj_launch),
            "graph": bool(args.graph),
        },
        "ray_steps": ray_steps,
        "rays": n_rays,
        "loss": loss,
        "fwd_ray_steps_per_s": ray_steps / (fwd_ms * 1e-3),
        "fwd_ms": fwd_ms,
        "fwd_kernel_ms": fwd_kernel_ms,
        "kernel_ms": {("mlp_forward_and_encode" if W.mlp is not None else "field_encode"): k_ms[0],
                      "trace_fwd_ckpt": k_ms[1], "render_loss": k_ms[2], "grad_zero": k_ms[3],
                      "trace_adjoint": k_ms[4], **({"mlp_backward_all_losses": k_ms[5]} if W.mlp is not None else {})},
        "roofline": {
            "kernel": "k_trace_adj (adjoint)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic,
            # the counted HBM bytes per launch over the launch time, against the HBM peak
            "hbm_frac": None if traffic is None else traffic / adj_s / PEAK_HBM_BYTES_PER_S,
            "flop_per_ray_step": flop_adj,
        },
        "roofline_fwd": {
            "kernel": "k_trace_fwd (forward, no checkpoints)",
            "bound": "alu",
            "achieved": flop_fwd * ray_steps / (fwd_kernel_ms * 1e-3) / 1e12,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": flop_fwd * ray_steps / (fwd_kernel_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
            "flop_per_ray_step": flop_fwd,
        },
    }
    if ceil is not None:
        vb = 4 if args.dtype == "f32" else 2
        gathers = {"roofline": (GATHER_ADJ_STEP, adj_s), "roofline_fwd": (GATHER_FWD_STEP, fwd_kernel_ms * 1e-3)}
        cg = ceil["gather_coherent_f32_tbps" if vb == 4 else "gather_coherent_16bit_tbps"]
        for key, (vals, t) in gathers.items():
            r = out[key]
            r["fma_ceiling_tflops"] = ceil["fma_fp32_tflops"]
            r["frac_of_fma_ceiling"] = r["achieved"] / ceil["fma_fp32_tflops"]
            # field values delivered to the lanes (algorithmic gather bytes) against the
            # coherent-gather ceiling measured on the same record layout and ray pattern
            if args.tracer == "nonlinear" or key == "roofline_fwd":
                per_step = (vals if not ql else 16) * vb
                got = per_step * ray_steps / t / 1e12
                r["vl1d"] = {"bytes_per_ray_step": per_step, "achieved_tbps": got, "ceiling_tbps": cg,
                             "frac": got / cg}
        if cnt is not None:
            # counter rates of this launch against the same counters of the ceiling kernels
            for key, g, t in (("roofline", "adj", adj_s), ("roofline_fwd", "fwd", fwd_kernel_ms * 1e-3)):
                r = out[key]
                m = {}
                if g + ".tcp_accesses" in cnt and "gather.tcp_accesses" in cnt:
                    a = cnt[g + ".tcp_accesses"] / t
                    c = cnt["gather.tcp_accesses"] / (ceil["ms"]["gather"] * 1e-3)
                    m["vl1d_accesses"] = {"achieved_per_s": a, "ceiling_per_s": c, "frac": a / c,
                                          "per_launch": cnt[g + ".tcp_accesses"]}
                if g + ".tcc_req" in cnt and "l2gather.tcc_req" in cnt:
                    a = cnt[g + ".tcc_req"] / t
                    c = cnt["l2gather.tcc_req"] / (ceil["ms"]["l2gather"] * 1e-3)
                    m["l2_requests"] = {"achieved_per_s": a, "ceiling_per_s": c, "frac": a / c,
                                        "per_launch": cnt[g + ".tcc_req"],
                                        "hit_rate": cnt.get(g + ".tcc_hit", 0.0) / max(cnt[g + ".tcc_req"], 1.0)}
                if g + ".hbm_read_bytes" in cnt and g + ".hbm_write_bytes" in cnt:
                    b = cnt[g + ".hbm_read_bytes"] + cnt[g + ".hbm_write_bytes"]
                    m["hbm"] = {"bytes_per_launch": b, "achieved_tbps": b / t / 1e12,
                                "ceiling_tbps": ceil["hbm_copy_tbps"], "frac": b / t / 1e12 / ceil["hbm_copy_tbps"],
                                "frac_of_peak": b / t / PEAK_HBM_BYTES_PER_S}
                r["memory"] = m
        out["ceilings"] = ceil
    if hasattr(W, "tuned"):
        out["config"]["autotune"] = W.tuned
    if mlp_info is not None:
        out["config"]["workload"] += (", temperatures from an MLP (64 units x %d tanh layers) at the 2,097,152 voxel "
                                      "centres, boundary loss on %d inlet points, Boussinesq PDE loss on %d "
                                      "collocation points" % (args.mlp_depth, args.boundary_points, args.pde_points))
        out["config"]["field"] = "mlp"
        out["mlp"] = mlp_info
    if not args.no_cpu and args.workload == "room1m" and W.mlp is None:
        out["cpu_baseline"], out["err"] = cpu_baseline_and_errors(args, W)
    if args.workload == "room256" and not args.no_cpu:
        out["err"] = subsample_errors(args, W)
    print(json.dumps(out), flush=True)


PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix (published)


def mlp_timing(args, W, cur):
    """HIP-event times of the network-field parts and the MFMA work of the grid forward."""
    import torch

    from paper_2509_14442_amd import api

    dims = W.descs[0].dims
    n = dims[0] * dims[1] * dims[2]
    D = args.mlp_depth
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    acc = [0.0] * 4
    for _ in range(args.steps):
        ev[0].record(cur)
        _, T = W.mlp.forward(grid=dims, want_out=False, T0=W.T0, T_in=W.T_in)
        ev[1].record(cur)
        seed = api.MLP.bos_seed(T, W.grads[0].reshape(-1), W.T0, W.T_in)
        W.mlp.backward(seed, grid=dims, dparams=W.dparams)
        ev[2].record(cur)
        out_b, _ = W.mlp.forward(W.pts_b)
        dL_b, _ = api.fit_seed(out_b, W.tgt_b, W.norms_b)
        W.mlp.backward(dL_b, W.pts_b, dparams=W.dparams)
        ev[3].record(cur)
        P = W.pde
        W.mlp.pde_loss(W.pts_c, P["Re"], P["Pe"], P["Ri"], P["L"], P["gamma"], dparams=W.dparams)
        ev[4].record(cur)
        torch.cuda.synchronize()
        for i in range(4):
            acc[i] += ev[i].elapsed_time(ev[i + 1])
    ms = [a / args.steps for a in acc]
    flop_point = 2 * (3 * 64 + (D - 1) * 64 * 64 + 64 * 5)
    achieved = flop_point * n / (ms[0] * 1e-3) / 1e12
    return {
        "grid_forward_ms": ms[0], "bos_chain_backward_ms": ms[1], "boundary_loss_ms": ms[2], "pde_loss_ms": ms[3],
        "params": int(W.mlp.params.numel()), "loss_boundary": float(W.loss_b[0]), "loss_pde": float(W.loss_pde[0]),
        "roofline_grid_forward": {"kernels": "k_mlp_forward_fused (%d layers)" % (D + 1), "bound": "mfma",
                                  "achieved": achieved, "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                                  "frac": achieved / PEAK_FP32_MFMA_TFLOPS, "flop_per_point": flop_point,
                                  "points": n},
    }


def _stored_delta(T, dtype, scale, offset):
    import oracle

    code = {"f32": oracle.CODE_F32, "f16": oracle.CODE_F16, "bf16": oracle.CODE_BF16}[dtype]
    return oracle.decode(oracle.encode(oracle.delta_from_temperature_f32(T), code, scale, offset), code, scale, offset)


def _gpu_subset(W, ids, dL, dL_ddir=None):
    """GPU forward + adjoint restricted to the pixel ids, with the given per-ray dL/d(u, v)
    (and dL/d(direction))."""
    import torch

    from paper_2509_14442_amd import api

    sub = api.Tracer([api.Scene(W.descs[0], W.fields[0], W.pat, torch.from_numpy(ids).cuda())], W.launch,
                     adjoint_launch=W.adj_launch)
    sub.forward()
    dd = None if dL_ddir is None else [torch.from_numpy(dL_ddir.astype("float32")).cuda()]
    g = sub.adjoint(dL_duv=[torch.from_numpy(dL.astype("float32")).cuda()], dL_ddir=dd)[0]
    torch.cuda.synchronize()
    return sub, g.cpu().numpy()


def cpu_baseline_and_errors(args, W):
    """The FP64 oracle (test infrastructure) timed on a bounded, evenly spread sample of the
    same rays; the GPU's outputs on that sample are compared with it."""
    import numpy as np

    import bos_inputs as bi
    import oracle

    oracle.build()
    desc = W.descs[0]
    p64 = W.pat_np.astype(np.float64)
    f = W.fields[0]
    FA = oracle.grid_field(_stored_delta(W.TA_np, args.dtype, f.scale, f.offset), desc.box_lo, desc.box_hi)
    FB = oracle.grid_field(_stored_delta(W.TB_np, args.dtype, f.scale, f.offset), desc.box_lo, desc.box_hi)

    spp = desc.spp

    radio = bool(desc.radiometry)

    def run(ids):
        tb = oracle.trace(FB, desc, ids)
        target = oracle.render_pixels(desc, p64, tb["uv"], tb["status"], tb["vdir"], tb["path"])["image"]
        t0 = time.perf_counter()
        fa = oracle.trace(FA, desc, ids)
        rp = oracle.render_pixels(desc, p64, fa["uv"], fa["status"], fa["vdir"], fa["path"])
        L, dL, dLd, dLp = oracle.loss_pixels(rp["image"], target, spp, rp["dI_duv"],
                                             rp["dI_ddir"] if radio else None, rp["dI_dpath"] if radio else None)
        g = oracle.adjoint(FA, desc, dL, ids, dL_ddir=dLd, dL_dpath=dLp)
        fa["dL_ddir"] = dLd
        return time.perf_counter() - t0, fa, dL, g

    # calibrate on a small sample, then size the sample for ~cpu_seconds of oracle work
    probe = bi.strided_tiles(desc.width, desc.height, 8, 256, 7)
    dt, fa, _, _ = run(probe)
    per_pixel = dt / max(len(probe), 1)
    n_target = int(args.cpu_seconds / max(per_pixel, 1e-9))
    total_tiles = ((desc.width + 7) // 8) * ((desc.height + 7) // 8)
    keep = max(1, int(total_tiles * 64 / max(n_target, 1)))
    ids = bi.strided_tiles(desc.width, desc.height, 8, keep, 3)
    dt, fa, dL, g_ref = run(ids)
    steps = int(fa["n_steps"].sum())
    cpu = {"value": steps / dt, "unit": "ray-steps/s", "cores": oracle.threads(), "kind": "oracle",
           "sample": f"{len(ids) * spp} rays ({spp} per pixel of 1 in {keep} 8x8 tiles of the 1024x1024 "
                     f"image), {steps} ray-steps, fwd+render+loss+adjoint in FP64, {dt:.1f} s"}
    tr = W.tracer
    rows = (np.arange(spp)[:, None] * (desc.width * desc.height) + ids[None, :]).ravel()
    uv = tr.uv[0].cpu().numpy().astype(np.float64)[rows]
    duv = tr.duv[0].cpu().numpy().astype(np.float64)[rows]
    ns = tr.n_steps[0].cpu().numpy()[rows]
    ok = np.isfinite(fa["uv"][:, 0])
    e_uv = np.sqrt(((uv[ok] - fa["uv"][ok]) ** 2).sum(1))
    e_duv = np.sqrt(((duv[ok] - fa["duv"][ok]) ** 2).sum(1))
    _, g = _gpu_subset(W, ids, dL, fa["dL_ddir"])
    if radio:
        # the GPU is given the oracle's (u, v) and direction seeds: compare with the same
        # map (the weight's path term is the oracle's own seed, outside the timed sample)
        g_ref = oracle.adjoint(FA, desc, dL, ids, dL_ddir=fa["dL_ddir"])
    l2 = float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))
    bound = 1e-3 * np.maximum(np.abs(g_ref), 1e-2 * np.abs(g_ref).max())
    err = {
        "sample_rays": int(len(rows)),
        "exit_err_max_m": float(e_uv.max()), "exit_err_rms_m": float(np.sqrt((e_uv ** 2).mean())),
        "exit_err_p99_m": float(np.percentile(e_uv, 99)),
        "deflection_err_max_m": float(e_duv.max()),
        "bos_displacement_rms_m": float(np.sqrt((fa["duv"][ok] ** 2).sum(1).mean())),
        "n_steps_mismatch": int((ns != fa["n_steps"]).sum()),
        "grad_rel_l2": l2,
        "grad_voxel_fail_frac": float(np.mean(np.abs(g - g_ref) > bound)),
    }
    if args.dtype != "f32":
        # storage + arithmetic: against the oracle on the unquantised field (bound 1e-5 m)
        FX = oracle.grid_field(oracle.delta_from_temperature(W.TA_np), desc.box_lo, desc.box_hi)
        fx = oracle.trace(FX, desc, ids)
        okx = ok & np.isfinite(fx["uv"][:, 0])
        e_x = np.sqrt(((uv[okx] - fx["uv"][okx]) ** 2).sum(1))
        err["vs_exact"] = {"offset": f.offset, "scale": f.scale, "exit_err_max_m": float(e_x.max()),
                           "exit_err_p99_m": float(np.percentile(e_x, 99)),
                           "bound_m": 1e-5, "meets_bound": bool(e_x.max() <= 1e-5),
                           "miss_factor": float(e_x.max() / 1e-5)}
    return cpu, err


def subsample_errors(args, W):
    """256x256x192 room: errors on a seeded 4096-ray subsample against the oracle on the dequantised
    field (arithmetic) and on the exact FP64 field (storage + arithmetic)."""
    import numpy as np

    import bos_inputs as bi
    import oracle

    oracle.build()
    desc = W.descs[0]
    f = W.fields[0]
    ids = bi.pixel_subset(desc.width * desc.height, 4096, 15)
    rows = (np.arange(desc.spp)[:, None] * (desc.width * desc.height) + ids[None, :]).ravel()
    rng = np.random.default_rng(16)
    lam = rng.standard_normal((len(rows), 2))
    _, g = _gpu_subset(W, ids, lam)
    uv = W.tracer.uv[0].cpu().numpy().astype(np.float64)[rows]
    out = {"sample_rays": int(len(rows)), "storage": storage(args), "offset": f.offset, "scale": f.scale}
    exact = oracle.delta_from_temperature(W.TA_np)
    deq = _stored_delta(W.TA_np, args.dtype, f.scale, f.offset)
    for name, delta in (("vs_dequantised", deq), ("vs_exact", exact)):
        F = oracle.grid_field(delta, desc.box_lo, desc.box_hi)
        ref = oracle.trace(F, desc, ids)
        ok = np.isfinite(ref["uv"][:, 0])
        e = np.sqrt(((uv[ok] - ref["uv"][ok]) ** 2).sum(1))
        g_ref = oracle.adjoint(F, desc, lam.astype(np.float32).astype(np.float64), ids)
        out[name] = {"exit_err_max_m": float(e.max()), "exit_err_rms_m": float(np.sqrt((e ** 2).mean())),
                     "grad_rel_l2": float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref))}
        if name == "vs_exact":
            out["bos_displacement_rms_m"] = float(np.sqrt((ref["duv"][ok] ** 2).sum(1).mean()))
    return out


if __name__ == "__main__":
    main()
