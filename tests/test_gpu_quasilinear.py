"""GPU parity of the quasi-linear tracer (forces on the straight entry line) against the
oracle's quasi-linear form: exit points <= 1e-6 m, images <= 1e-5, gradients
rel-L2 < 1e-3 (same tolerances as the nonlinear form), branch-locked differences on
voxels that include the entry layer, launch shapes that agree, and the full 1M-ray room
in the benchmark's launch configuration. The quasi-linear exit points are also compared
with the nonlinear ones, the approximation the paper makes."""

import numpy as np
import pytest
import torch

import bos_inputs as bi
import oracle
from _common import bench_tuned, exit_error, grad_errors, oracle_forward, room_workload, stored_delta, unit_box_workload
from paper_2509_14442_amd import api
from test_gpu_forward import DEV, NOT_OFF, _np

pytestmark = pytest.mark.gpu

QL = oracle.oracle.TRACER_QUASILINEAR


def _ql(w):
    w.scene = w.scene.replace(tracer=QL)
    return w


def _tracer(w, launch=None, adj_launch=None, ids=None):
    field = api.Field.from_temperature(torch.from_numpy(w.T32).to(DEV), "f32")
    ids_t = None if ids is None else torch.from_numpy(ids).to(DEV)
    sc = api.Scene(w.scene, field, torch.from_numpy(w.pattern32).to(DEV), ids_t)
    return api.Tracer([sc], launch, adjoint_launch=adj_launch)


def _check_forward(w, tr, max_step_mismatch=0):
    _, ref = oracle_forward(w, stored_delta(w.T32))
    ns, st = _np(tr.n_steps[0]), _np(tr.status[0])
    assert (ns != ref["n_steps"]).sum() <= max_step_mismatch
    assert np.array_equal(st & NOT_OFF, ref["status"] & NOT_OFF)
    ok = np.isfinite(ref["uv"][:, 0])
    assert np.array_equal(ok, np.isfinite(_np(tr.uv[0])[:, 0]))
    assert exit_error(_np(tr.uv[0])[ok], ref["uv"][ok]).max() <= 1e-6
    assert exit_error(_np(tr.duv[0])[ok], ref["duv"][ok]).max() <= 1e-6
    assert np.abs(_np(tr.image[0]) - ref["image"]).max() <= 1e-5
    return ref


def test_ql_forward_unit_box_and_room():
    w = _ql(unit_box_workload())
    tr = _tracer(w)
    tr.forward().render()
    torch.cuda.synchronize()
    _check_forward(w, tr)
    w = _ql(room_workload((128, 128, 128), 256, 256, seed=2))
    tr = _tracer(w)
    tr.forward().render()
    torch.cuda.synchronize()
    ref = _check_forward(w, tr, max_step_mismatch=2)
    # the approximation itself: quasi-linear against nonlinear exit points (oracle)
    w_nl = room_workload((128, 128, 128), 256, 256, seed=2)
    _, nl = oracle_forward(w_nl, stored_delta(w_nl.T32))
    ok = np.isfinite(nl["uv"][:, 0]) & np.isfinite(ref["uv"][:, 0])
    gap = exit_error(ref["uv"][ok], nl["uv"][ok])
    disp = np.sqrt((nl["duv"][ok] ** 2).sum(1))
    print(f"quasi-linear vs nonlinear exit: rms {np.sqrt((gap ** 2).mean()):.2e} m, max {gap.max():.2e} m; "
          f"BOS displacement rms {np.sqrt((disp ** 2).mean()):.2e} m")
    assert np.sqrt((gap ** 2).mean()) < 1e-3 * np.sqrt((disp ** 2).mean())


@pytest.mark.parametrize("room", [False, True])
def test_ql_adjoint_matches_oracle(room):
    if room:
        w = _ql(room_workload((64, 64, 48), 256, 256, seed=3))
        rng = np.random.default_rng(15)
        ids = np.sort(rng.choice(256 * 256, 4096, replace=False)).astype(np.int32)
    else:
        w = _ql(unit_box_workload())
        rng = np.random.default_rng(16)
        ids = None
    n = w.scene.n_pixels if ids is None else len(ids)
    lam = rng.standard_normal((n, 2)).astype(np.float32)
    tr = _tracer(w, ids=ids)
    tr.forward()
    g = _np(tr.adjoint(dL_duv=[torch.from_numpy(lam).to(DEV)])[0])
    F = oracle.grid_field(stored_delta(w.T32), w.scene.box_lo, w.scene.box_hi)
    g_ref = oracle.adjoint(F, w.scene, lam.astype(np.float64), ids)
    l2, frac = grad_errors(g, g_ref)
    assert l2 < 1e-3 and frac < 5e-3, (l2, frac)


def test_ql_adjoint_sparse_rays_every_lane_in_its_own_cell():
    """Rays 3-10 cells apart (24 x 24 camera, 240 x 240 x 180 room): the quasi-linear
    adjoint's parked sums and 32-slot cell cache under dozens of cells per reduction."""
    w = _ql(room_workload((240, 240, 180), 24, 24, seed=7, max_steps=800, pat=256))
    lam = np.random.default_rng(9).standard_normal((24 * 24, 2)).astype(np.float32)
    tr = _tracer(w)
    tr.forward()
    g = _np(tr.adjoint(dL_duv=[torch.from_numpy(lam).to(DEV)])[0])
    F = oracle.grid_field(stored_delta(w.T32), w.scene.box_lo, w.scene.box_hi)
    g_ref = oracle.adjoint(F, w.scene, lam.astype(np.float64))
    l2, frac = grad_errors(g, g_ref)
    assert l2 < 1e-3 and frac < 5e-3, (l2, frac)


def test_ql_adjoint_locked_differences_including_entry_layer():
    w = _ql(unit_box_workload(40, 40))
    T2 = bi.temperature_grid(bi.plume_unit_box(2), w.scene.box_lo, w.scene.box_hi, w.scene.dims)
    _, r2 = oracle_forward(w, stored_delta(T2.astype(np.float32)))
    target = r2["image"].astype(np.float32)
    tr = _tracer(w)
    tr.forward().render([torch.from_numpy(target).to(DEV)])
    g = _np(tr.adjoint()[0])
    F, ref = oracle_forward(w, stored_delta(w.T32))
    _, dL = oracle.loss(ref["image"], target.astype(np.float64), ref["dI"])
    g_or = oracle.adjoint(F, w.scene, dL)
    gmax = np.abs(g).max()
    cand = np.flatnonzero(np.abs(g_or) > 1e-2 * np.abs(g_or).max())  # voxels chosen by the oracle
    nx, ny, _ = w.scene.dims
    entry = cand[(cand // nx) % ny == 0]
    rng = np.random.default_rng(23)
    vox = np.concatenate([rng.choice(cand, 12, replace=False), rng.choice(entry, 4, replace=False)])
    pat = w.pattern32.astype(np.float64)
    fd1 = oracle.fd_voxels(F, w.scene, pat, target.astype(np.float64), vox, h=1e-7)
    fd2 = oracle.fd_voxels(F, w.scene, pat, target.astype(np.float64), vox, h=2e-7)
    fd = (4.0 * fd1 - fd2) / 3.0
    assert np.allclose(g.ravel()[vox], fd, rtol=1e-3, atol=1e-3 * gmax), np.c_[g.ravel()[vox], fd]


def test_ql_launch_shapes_agree():
    w = _ql(room_workload((48, 40, 32), 96, 80, seed=4))
    rng = np.random.default_rng(1)
    lam = torch.from_numpy(rng.standard_normal((96 * 80, 2)).astype(np.float32)).to(DEV)
    outs = []
    for launch in (None, api.make_launch((8, 8), 4, persistent=True), api.make_launch((16, 4), 1)):
        tr = _tracer(w, launch, launch)
        tr.forward()
        outs.append((tr.uv[0].clone(), _np(tr.adjoint(dL_duv=[lam])[0])))
    for uv, g in outs[1:]:
        assert torch.equal(uv, outs[0][0])
        assert np.linalg.norm(g - outs[0][1]) <= 1e-5 * np.linalg.norm(outs[0][1])


def test_ql_room_1m_in_bench_configuration():
    w = _ql(room_workload((128, 128, 128), 1024, 1024, seed=3))
    field = api.Field.from_temperature(torch.from_numpy(w.T32).to(DEV), "f32")
    fwd, adj, k = bench_tuned([api.Scene(w.scene, field, torch.from_numpy(w.pattern32).to(DEV))])
    w.scene = w.scene.replace(ckpt_stride=k)
    tr = _tracer(w, fwd, adj)
    tr.forward()
    uv = _np(tr.uv[0])
    sample = bi.pixel_subset(1024 * 1024, 4096, 15)
    w.pixel_ids = sample
    F, ref = oracle_forward(w, stored_delta(w.T32))
    ok = np.isfinite(ref["uv"][:, 0])
    assert exit_error(uv[sample][ok], ref["uv"][ok]).max() <= 1e-6
    rng = np.random.default_rng(22)
    lam = (rng.standard_normal((4096, 2)) * 1e-3).astype(np.float32)
    trs = _tracer(w, fwd, adj, ids=sample)
    trs.forward()
    g = _np(trs.adjoint(dL_duv=[torch.from_numpy(lam).to(DEV)])[0])
    g_ref = oracle.adjoint(F, w.scene, lam.astype(np.float64), sample)
    l2, frac = grad_errors(g, g_ref)
    assert l2 < 1e-3 and frac < 5e-3, (l2, frac)
