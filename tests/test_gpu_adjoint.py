"""GPU parity of the loss, dL/d(u, v) and the checkpointed adjoint against the oracle.

Gradient tolerance: ||g - g_ref||_2 / ||g_ref||_2 < 1e-3 over the compared voxels, and
per voxel |g - g_ref| <= 1e-3 max(|g_ref|, 1e-2 ||g_ref||_inf) for all but a small
fraction (cells chosen differently by FP32 and FP64 arithmetic within ~1e-9 m of a face).
"""

import numpy as np
import pytest
import torch

import oracle
from _common import unit_box_workload, grad_errors, oracle_forward, room_workload, stored_delta
from paper_2509_14442_amd import api
from test_gpu_forward import DEV, _np

pytestmark = pytest.mark.gpu


def _target(w, seed_field):
    """Measured image: the oracle's render of a second field, stored as float32."""
    _, ref = oracle_forward(w, stored_delta(seed_field))
    return ref["image"].astype(np.float32)


def _gpu_loss_and_grad(w, target, launch=None, ckpt=16, dL_duv=None):
    T = torch.from_numpy(w.T32).to(DEV)
    field = api.Field.from_temperature(T, "f32")
    pat = torch.from_numpy(w.pattern32).to(DEV)
    ids = None if w.pixel_ids is None else torch.from_numpy(w.pixel_ids).to(DEV)
    sc = api.Scene(w.scene, field, pat, ids, ckpt_stride=ckpt)
    tr = api.Tracer([sc], launch=launch)
    tr.forward().render([torch.from_numpy(target).to(DEV)])
    lam = None if dL_duv is None else [torch.from_numpy(dL_duv).to(DEV)]
    g = tr.adjoint(dL_duv=lam)[0]
    torch.cuda.synchronize()
    return tr, _np(g)


def _oracle_loss_and_grad(w, target, dL_duv=None):
    F, ref = oracle_forward(w, stored_delta(w.T32))
    L, dL = oracle.loss(ref["image"], target.astype(np.float64), ref["dI"])
    lam = dL if dL_duv is None else dL_duv.astype(np.float64)
    g = oracle.adjoint(F, w.scene, lam, w.pixel_ids)
    return L, dL, g, F


def test_loss_and_dl_duv_unit_box():
    w = unit_box_workload()
    from bos_inputs import plume_unit_box, temperature_grid
    T2 = temperature_grid(plume_unit_box(2), w.scene.box_lo, w.scene.box_hi, w.scene.dims).astype(np.float32)
    target = _target(w, T2)
    tr, _ = _gpu_loss_and_grad(w, target)
    L, dL, _, _ = _oracle_loss_and_grad(w, target)
    assert float(tr.loss[0]) == pytest.approx(L, rel=1e-5)
    got = _np(tr.dL_duv[0])
    scale = np.abs(dL).max()
    assert np.abs(got - dL).max() <= 1e-4 * scale


@pytest.mark.parametrize("ckpt", [1, 3, 4, 6, 8, 16, 32])
def test_adjoint_unit_box_matches_oracle(ckpt):
    w = unit_box_workload()
    from bos_inputs import plume_unit_box, temperature_grid
    T2 = temperature_grid(plume_unit_box(2), w.scene.box_lo, w.scene.box_hi, w.scene.dims).astype(np.float32)
    target = _target(w, T2)
    # one dL/d(u, v) for both sides: the oracle's, as float32
    _, dL, _, _ = _oracle_loss_and_grad(w, target)
    lam = dL.astype(np.float32)
    _, g = _gpu_loss_and_grad(w, target, ckpt=ckpt, dL_duv=lam)
    _, _, g_ref, _ = _oracle_loss_and_grad(w, target, dL_duv=lam)
    l2, frac = grad_errors(g, g_ref)
    assert l2 < 1e-3, (l2, frac)
    assert frac < 2e-3, (l2, frac)


def test_adjoint_room_subset_matches_oracle():
    w = room_workload((64, 64, 48), 256, 256, seed=3)
    rng = np.random.default_rng(15)
    w.pixel_ids = np.sort(rng.choice(256 * 256, 4096, replace=False)).astype(np.int32)
    lam = rng.standard_normal((4096, 2)).astype(np.float32)
    _, g = _gpu_loss_and_grad(w, np.zeros(4096, np.float32), dL_duv=lam)
    _, _, g_ref, _ = _oracle_loss_and_grad(w, np.zeros(4096, np.float32), dL_duv=lam)
    l2, frac = grad_errors(g, g_ref)
    assert l2 < 1e-3, (l2, frac)
    assert frac < 5e-3, (l2, frac)


_SPARSE = {}


def _sparse_reference():
    """A 24 x 24 camera on a 240 x 240 x 180 room and one dL/d(u, v); the oracle's gradient."""
    if not _SPARSE:
        w = room_workload((240, 240, 180), 24, 24, seed=7, max_steps=800, pat=256)
        lam = np.random.default_rng(8).standard_normal((24 * 24, 2)).astype(np.float32)
        _, _, g_ref, _ = _oracle_loss_and_grad(w, np.zeros(24 * 24, np.float32), dL_duv=lam)
        _SPARSE.update(w=w, lam=lam, g_ref=g_ref)
    return _SPARSE["w"], _SPARSE["lam"], _SPARSE["g_ref"]


@pytest.mark.parametrize("ckpt", [1, 3, 4, 6, 8])
def test_adjoint_sparse_rays_every_lane_in_its_own_cell(ckpt):
    """Rays 3-10 cells apart: the 64 rays of a tile sit in different cells, so one
    wavefront reduction follows another for dozens of cells at a time, and the
    wavefront's 32-slot cache of cell totals fills and writes slots out within a chunk.
    Every adjoint form (stored, recording, replay; with and without parked sums) against
    the oracle."""
    w, lam, g_ref = _sparse_reference()
    _, g = _gpu_loss_and_grad(w, np.zeros(24 * 24, np.float32), ckpt=ckpt, dL_duv=lam)
    l2, frac = grad_errors(g, g_ref)
    assert l2 < 1e-3 and frac < 5e-3, (l2, frac)


@pytest.mark.parametrize("ckpt", [16, 3, 4])
def test_adjoint_persistent_and_tiles_agree(ckpt):
    w = room_workload((48, 40, 32), 96, 80, seed=4)
    rng = np.random.default_rng(1)
    lam = rng.standard_normal((96 * 80, 2)).astype(np.float32)
    _, g0 = _gpu_loss_and_grad(w, np.zeros(96 * 80, np.float32), ckpt=ckpt, dL_duv=lam)
    for launch in (api.make_launch((8, 8), 4, persistent=True, blocks_per_cu=2), api.make_launch((16, 4), 1)):
        _, g1 = _gpu_loss_and_grad(w, np.zeros(96 * 80, np.float32), launch=launch, ckpt=ckpt, dL_duv=lam)
        assert np.linalg.norm(g1 - g0) <= 1e-5 * np.linalg.norm(g0)


def test_adjoint_against_locked_finite_differences():
    w = unit_box_workload(32, 32)
    from bos_inputs import plume_unit_box, temperature_grid
    T2 = temperature_grid(plume_unit_box(2), w.scene.box_lo, w.scene.box_hi, w.scene.dims).astype(np.float32)
    target = _target(w, T2)
    tr, g = _gpu_loss_and_grad(w, target)
    _, _, g_or, F = _oracle_loss_and_grad(w, target)
    rng = np.random.default_rng(13)
    cand = np.flatnonzero(np.abs(g_or) > 1e-2 * np.abs(g_or).max())  # voxels chosen by the oracle
    vox = rng.choice(cand, 16, replace=False)
    fd = oracle.fd_voxels(F, w.scene, w.pattern32.astype(np.float64), target.astype(np.float64), vox, h=1e-7)
    ref = g.ravel()[vox]
    assert np.allclose(ref, fd, rtol=1e-3, atol=1e-3 * np.abs(g).max()), np.c_[ref, fd]


def test_bos_loss_autograd():
    """torch.autograd through BOSLoss: the loss equals the oracle's and the gradient
    d(3 L)/d(eta - 1) equals 3 x the tracer's adjoint and the oracle's."""
    w = unit_box_workload(48, 48)
    from bos_inputs import plume_unit_box, temperature_grid
    T2 = temperature_grid(plume_unit_box(2), w.scene.box_lo, w.scene.box_hi, w.scene.dims).astype(np.float32)
    target = _target(w, T2)
    d32 = oracle.delta_from_temperature_f32(w.T32)
    delta = torch.from_numpy(d32.astype(np.float32)).to(DEV).requires_grad_(True)
    field = api.Field.from_delta(delta.detach(), "f32")
    sc = api.Scene(w.scene, field, torch.from_numpy(w.pattern32).to(DEV))
    tr = api.Tracer([sc])
    tgt = torch.from_numpy(target).to(DEV)
    L = api.bos_loss(delta, tr, tgt)
    (3.0 * L).backward()
    torch.cuda.synchronize()
    L_ref, dL, g_ref, _ = _oracle_loss_and_grad(w, target)
    assert float(L) == pytest.approx(L_ref, rel=1e-5)
    g = _np(delta.grad).astype(np.float64) / 3.0
    l2, frac = grad_errors(g, g_ref)
    assert l2 < 1e-3, (l2, frac)
