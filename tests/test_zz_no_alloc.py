"""rbos_trace_adjoint_noalloc (no device allocation: its scratch is the library's static
device array) against rbos_trace_adjoint with a caller workspace, on two calls in a row,
the second with a smaller input, so the second call runs on the scratch the first one
left behind. Both calls go through the C ABI (ctypes)."""

import numpy as np
import pytest
import torch

import oracle
from _common import grad_errors, room_workload, stored_delta
from paper_2509_14442_amd import api

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _run(w, target, launch, ckpt):
    """Forward + render + loss, then the gradient from both adjoint entry points."""
    print(f"noalloc case: dims {w.scene.dims} camera {w.scene.width}x{w.scene.height} ckpt {ckpt} "
          f"persistent {launch.persistent}", flush=True)
    field = api.Field.from_temperature(torch.from_numpy(w.T32).to(DEV), "f32")
    pat = torch.from_numpy(w.pattern32).to(DEV)
    tr = api.Tracer([api.Scene(w.scene, field, pat, ckpt_stride=ckpt)], launch)
    tr.forward().render([torch.from_numpy(target).to(DEV)])
    g_ws = tr.adjoint()[0]
    g_na = tr.adjoint(noalloc=True)[0]
    torch.cuda.synchronize()
    return tr, g_ws.cpu().numpy(), g_na.cpu().numpy()


def _target(w, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, w.scene.width * w.scene.height).astype(np.float32)


def test_noalloc_adjoint_matches_workspace_adjoint_twice():
    big = room_workload(dims=(64, 64, 48), width=200, height=152, seed=2, ckpt=6, pat=256)
    small = room_workload(dims=(32, 32, 24), width=72, height=40, seed=3, ckpt=8, pat=256)
    persistent = api.make_launch((8, 8), 2, True, 0)
    grid = api.make_launch((16, 4), 4, False, 0)

    # first call: persistent launch (queues, tile costs and order in the scratch)
    _, g_ws, g_na = _run(big, _target(big, 21), persistent, 6)
    scale = np.abs(g_ws).max()
    assert scale > 0
    assert np.abs(g_na - g_ws).max() <= 1e-12 * scale

    # second call, smaller: the scratch still holds the first call's table and order
    for launch in (persistent, grid):
        tr, g_ws, g_na = _run(small, _target(small, 22), launch, 8)
        scale = np.abs(g_ws).max()
        assert scale > 0
        assert np.abs(g_na - g_ws).max() <= 1e-12 * scale

    # and the small case against the FP64 oracle (gradient bar of the adjoint parity tests)
    F = oracle.grid_field(stored_delta(small.T32), small.scene.box_lo, small.scene.box_hi)
    lam = tr.dL_duv[0].cpu().numpy().astype(np.float64)
    g_ref = oracle.adjoint(F, small.scene, lam)
    l2, frac = grad_errors(g_na, g_ref)
    assert l2 < 1e-3 and frac < 1e-3, (l2, frac)
