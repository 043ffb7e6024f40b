"""Ceilings of the GPU at hand, measured with the microbenchmarks of librbos_ceilings.so
(include/rbos_ceilings.h): the tracer kernels' rooflines are stated against these next
to the published peaks. Argument marshalling and HIP-event timing only."""

from __future__ import annotations

import ctypes as C
import os
from typing import Dict

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbos_ceilings.so")

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_14442_amd.build`")
        lib = C.CDLL(LIB_PATH)
        P, I = C.c_void_p, C.c_int
        lib.ceil_gather_coherent.argtypes = [P, I, I, I, I, I, I, I, P, P]
        lib.ceil_gather_scattered.argtypes = [P, I, I, I, I, P, P]
        lib.ceil_fma.argtypes = [P, I, I, P]
        lib.ceil_atomic_f64.argtypes = [P, I, I, I, I, I, P]
        lib.ceil_copy.argtypes = [P, P, C.c_size_t, I, P]
        for f in (lib.ceil_gather_coherent, lib.ceil_gather_scattered, lib.ceil_fma, lib.ceil_atomic_f64,
                  lib.ceil_copy):
            f.restype = C.c_int
        _lib = lib
    return _lib


def _time_ms(launch, reps: int = 5, warmup: int = 2) -> float:
    """Median duration (ms) of one launch, HIP events on the stream it is launched on."""
    stream = torch.cuda.current_stream()
    s = C.c_void_p(stream.cuda_stream)
    for _ in range(warmup):
        if launch(s) != 0:
            raise RuntimeError("ceiling kernel launch failed")
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        launch(s)
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def measure(dev="cuda:0", reps: int = 5) -> Dict[str, float]:
    """Measured ceilings (rates per second) and the shapes they were measured on."""
    lib = load()
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    out: Dict[str, float] = {}
    times: Dict[str, float] = {}  # ms per launch of each ceiling kernel

    # plain FP32 FMA rate: 8 wavefronts per SIMD on every compute unit
    blocks, iters = 16 * n_cu, 4096
    buf = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    ms = _time_ms(lambda s: lib.ceil_fma(C.c_void_p(buf.data_ptr()), blocks, iters, s), reps)
    out["fma_fp32_tflops"] = blocks * 256 * iters * 32 / (ms * 1e-3) / 1e12
    times["fma"] = ms

    # HBM stream copy: 1 GiB read + 1 GiB written
    nbytes = 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    ms = _time_ms(lambda s: lib.ceil_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), nbytes,
                                          4 * n_cu * 8, s), reps)
    out["hbm_copy_tbps"] = 2 * nbytes / (ms * 1e-3) / 1e12
    times["copy"] = ms
    del a, b

    # coherent cell-record gathers over the headline field's record grid (129^3 cells
    # with the apron), 1024 x 1024 rays, 256 steps of three samples
    px = py = pz = 129
    w = h = 1024
    steps = 256
    for rec_bytes, key in ((32, "gather_coherent_f32_tbps"), (16, "gather_coherent_16bit_tbps")):
        recs = torch.rand(px * py * pz * rec_bytes // 4, dtype=torch.float32, device=dev)
        o = torch.empty((w // 8) * (h // 8) * 64, dtype=torch.float32, device=dev)
        ms = _time_ms(lambda s: lib.ceil_gather_coherent(C.c_void_p(recs.data_ptr()), rec_bytes, px, py, pz, w, h,
                                                         steps, C.c_void_p(o.data_ptr()), s), reps)
        out[key] = w * h * steps * 3 * rec_bytes / (ms * 1e-3) / 1e12
        times["gather" if rec_bytes == 32 else "gather16"] = ms
        del recs, o

    # scattered 32-byte gathers within 2 MiB (L2-resident, a separate line per access)
    # and within 1 GiB (beyond the MALL)
    for log2_n, key in ((16, "gather_scattered_l2_f32_tbps"), (25, "gather_scattered_hbm_f32_tbps")):
        recs = torch.rand((1 << log2_n) * 8, dtype=torch.float32, device=dev)
        blocks, iters = 16 * n_cu, 256
        o = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
        ms = _time_ms(lambda s: lib.ceil_gather_scattered(C.c_void_p(recs.data_ptr()), 32, log2_n, blocks, iters,
                                                          C.c_void_p(o.data_ptr()), s), reps)
        out[key] = blocks * 256 * iters * 32 / (ms * 1e-3) / 1e12
        times["l2gather" if log2_n == 16 else "hbmgather"] = ms
        del recs, o

    # FP64 atomic adds into a 128^3 gradient, 8 lanes per cell
    g = torch.zeros((128, 128, 128), dtype=torch.float64, device=dev)
    blocks, iters = 16 * n_cu, 64
    ms = _time_ms(lambda s: lib.ceil_atomic_f64(C.c_void_p(g.data_ptr()), 128, 128, 128, blocks, iters, s), reps)
    out["atomic_f64_per_s"] = blocks * 256 * iters / (ms * 1e-3)
    times["atomic"] = ms
    del g
    torch.cuda.synchronize()
    out["ms"] = times
    return out
