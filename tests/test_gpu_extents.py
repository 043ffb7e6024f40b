"""GPU parity at the largest voxel count per axis (448): one long axis per case, the others
short, so that cell keys, record strides and the gradient's voxel index reach their
largest values on that axis while the oracle still traces every ray in well under a
second. Rays cross ~900-1200 cells and take up to ~1200 Sharma steps (many checkpoint
segments).

Tolerances as in the other forward and adjoint tests: wall exit within 1e-6 m, gradient
rel-L2 < 1e-3 with per-voxel agreement for all but a small fraction of voxels.
"""

import numpy as np
import pytest
import torch

import oracle
from _common import grad_errors, oracle_forward, room_workload, stored_delta
from paper_2509_14442_amd import api
from test_gpu_forward import DEV, _compare_forward, _np, gpu_trace

pytestmark = pytest.mark.gpu

MAX_DIM = 448


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_longest_axis_forward_and_adjoint(axis):
    dims = [6, 5, 7]
    dims[axis] = MAX_DIM
    w = room_workload(tuple(dims), 24, 24, seed=20 + axis, max_steps=1400, ckpt=16, pat=256)
    tr = gpu_trace(w, ckpt=True)
    _, _, ref = _compare_forward(w, tr, max_step_mismatch=2)
    ns = ref["n_steps"]
    print(f"dims {tuple(dims)}: steps per ray max {ns.max()}, mean {ns.mean():.0f}")
    assert ns.max() > 800  # long in-box paths

    rng = np.random.default_rng(30 + axis)
    lam = rng.standard_normal((24 * 24, 2)).astype(np.float32)
    g = _np(tr.adjoint(dL_duv=[torch.from_numpy(lam).to(DEV)])[0])
    F = oracle.grid_field(stored_delta(w.T32), w.scene.box_lo, w.scene.box_hi)
    g_ref = oracle.adjoint(F, w.scene, lam.astype(np.float64))
    l2, frac = grad_errors(g, g_ref)
    print(f"dims {tuple(dims)}: gradient rel-L2 {l2:.2e}, voxels off {frac:.1e}")
    assert l2 < 1e-3 and frac < 5e-3, (l2, frac)
    # the far end of the long axis receives gradient
    far = np.take(np.abs(g_ref), range(MAX_DIM - 16, MAX_DIM), axis=2 - axis)
    assert far.max() > 0
    # the recording adjoint (strides 4 and 3: cell keys of the samples kept from the
    # replay), the second with the field stored as x-pairs
    pat = torch.from_numpy(w.pattern32).to(DEV)
    for k, layout in ((4, "cell"), (3, "xpair")):
        field = api.Field.from_temperature(torch.from_numpy(w.T32).to(DEV), "f32")
        if layout != "cell":
            field = field.relayout(layout)
        trk = api.Tracer([api.Scene(w.scene.replace(ckpt_stride=k), field, pat)], checkpoints=True)
        trk.forward()
        assert torch.equal(trk.uv[0], tr.uv[0])
        gk = _np(trk.adjoint(dL_duv=[torch.from_numpy(lam).to(DEV)])[0])
        l2, frac = grad_errors(gk, g_ref)
        print(f"dims {tuple(dims)}, stride {k}, {layout}: gradient rel-L2 {l2:.2e}, voxels off {frac:.1e}")
        assert l2 < 1e-3 and frac < 5e-3, (k, layout, l2, frac)
