"""GPU parity of the field encoding, the forward trace and the render against the oracle.

Tolerances: exit point (wall-plane distance) <= 1e-6 m for FP32 storage. The image is
bilinear in the hit: |dI| <= |grad I| |d(u, v)| + FP32 rounding; with texels of >= 6 mm
and unit contrast, a 1e-8 m hit difference moves I by < 2e-6, so images are compared at
1e-5 absolute."""

import numpy as np
import pytest
import torch

import oracle
from _common import (CODES, RHO0G, T0, unit_box_workload, exit_error, expected_scale, oracle_forward,
                     room_workload, stored_delta)
from paper_2509_14442_amd import api

pytestmark = pytest.mark.gpu

DEV = "cuda"
NOT_OFF = np.uint8(0xFF ^ oracle.RAY_OFF_PATTERN)


def gpu_trace(w, dtype="f32", scale=1.0, offset=0.0, pixel_ids=None, ckpt=False, launch=None, render=True):
    T = torch.from_numpy(w.T32).to(DEV)
    field = api.Field.from_temperature(T, dtype, scale, offset)
    pat = torch.from_numpy(w.pattern32).to(DEV)
    if pixel_ids is None:
        pixel_ids = w.pixel_ids
    ids = None if pixel_ids is None else torch.from_numpy(pixel_ids).to(DEV)
    sc = api.Scene(w.scene, field, pat, ids)
    tr = api.Tracer([sc], launch=launch, checkpoints=ckpt)
    tr.forward()
    if render:
        tr.render()
    torch.cuda.synchronize()
    return tr


def _np(t):
    return t.detach().cpu().numpy()


def _expected_records(codes: np.ndarray) -> np.ndarray:
    """Cell records of the padded grid from per-voxel codes [nz][ny][nx]: record (k, j, i)
    for cells -1 .. n-1 holds corner c = a + 2b + 4z at voxel clamp(i + a) etc."""
    nz, ny, nx = codes.shape
    out = np.empty((nz + 1, ny + 1, nx + 1, 8), codes.dtype)
    ix, iy, iz = np.arange(-1, nx), np.arange(-1, ny), np.arange(-1, nz)
    for c in range(8):
        a, b, z = c & 1, (c >> 1) & 1, c >> 2
        X = np.clip(ix + a, 0, nx - 1)
        Y = np.clip(iy + b, 0, ny - 1)
        Z = np.clip(iz + z, 0, nz - 1)
        out[..., c] = codes[Z][:, Y][:, :, X]
    return out


@pytest.mark.parametrize("dtype,offset", [("f32", 0.0), ("f16", 0.0), ("f16", 2.7e-4), ("bf16", 0.0),
                                          ("bf16", 2.7e-4)])
def test_field_codes_bit_exact(dtype, offset):
    w = room_workload((37, 23, 19), 8, 8, seed=5)
    T = torch.from_numpy(w.T32).to(DEV)
    field = api.Field.from_temperature(T, dtype, None, offset)
    torch.cuda.synchronize()
    nx, ny, nz = field.dims
    got = _np(field.buf).view(np.uint32 if dtype == "f32" else np.uint16).reshape(nz + 1, ny + 1, nx + 1, 8)
    scale = expected_scale(w.T32, dtype, offset)
    assert field.scale == scale
    d32 = oracle.delta_from_temperature_f32(w.T32, RHO0G, T0)
    ref = oracle.encode(d32, CODES[dtype], scale, offset)
    if dtype == "f32":
        # FP32 records hold the trilinear coefficients of each cell, differences of the
        # corner codes rounded to binary32 in the documented order
        q = _expected_records(ref).astype(np.float32)
        d1, d3, d5, d7 = q[..., 1] - q[..., 0], q[..., 3] - q[..., 2], q[..., 5] - q[..., 4], q[..., 7] - q[..., 6]
        C = np.empty_like(q)
        C[..., 0], C[..., 1] = q[..., 0], d1
        C[..., 2], C[..., 4] = q[..., 2] - q[..., 0], q[..., 4] - q[..., 0]
        C[..., 3], C[..., 5] = d3 - d1, d5 - d1
        C[..., 6] = (q[..., 6] - q[..., 4]) - C[..., 2]
        C[..., 7] = (d7 - d5) - C[..., 3]
        assert np.array_equal(got, C.view(np.uint32))
    else:
        assert np.array_equal(got, _expected_records(ref))
    if dtype != "f32":
        q = oracle.decode(ref, CODES[dtype], scale, 0.0) * scale
        assert np.abs(q).max() <= 2 ** 14  # scale keeps the codes in range


def _compare_forward(w, tr, tol_exit=1e-6, max_step_mismatch=0):
    _, ref = oracle_forward(w, stored_delta(w.T32))
    ns, st = _np(tr.n_steps[0]), _np(tr.status[0])
    mism = np.flatnonzero(ns != ref["n_steps"])
    assert len(mism) <= max_step_mismatch, (len(mism), mism[:10])
    assert np.array_equal(st & NOT_OFF, ref["status"] & NOT_OFF)
    ok = np.isfinite(ref["uv"][:, 0])
    assert np.array_equal(ok, np.isfinite(_np(tr.uv[0])[:, 0]))
    err = exit_error(_np(tr.uv[0])[ok], ref["uv"][ok])
    derr = exit_error(_np(tr.duv[0])[ok], ref["duv"][ok])
    assert err.max() <= tol_exit, err.max()
    assert derr.max() <= tol_exit, derr.max()
    img = _np(tr.image[0])
    assert np.abs(img - ref["image"]).max() <= 1e-5
    assert np.array_equal(_np(tr.status[0]), ref["status_r"])
    return err, derr, ref


def test_forward_unit_box_full():
    w = unit_box_workload()
    tr = gpu_trace(w)
    err, derr, ref = _compare_forward(w, tr)
    # deflection accuracy far below the tolerance (double-float geometry, exact base)
    assert derr.max() < 1e-8, derr.max()
    assert (ref["status"] & oracle.RAY_MISSED_BOX).sum() > 0  # some rays miss the box


def test_forward_room_512():
    w = room_workload()
    tr = gpu_trace(w)
    err, derr, ref = _compare_forward(w, tr, max_step_mismatch=5)
    assert derr.max() < 1e-7, derr.max()
    # a ray whose step count differs (a state within rounding of a box face) moves the
    # total by at most one step per mismatched ray
    ns = _np(tr.n_steps[0]).astype(np.int64)
    mism = int((ns != ref["n_steps"]).sum())
    assert abs(int(ns.sum()) - int(ref["n_steps"].sum())) <= mism <= 5


def test_forward_ragged_camera_and_tiles():
    w = unit_box_workload(67, 45)
    for tile in ((8, 8), (16, 4), (64, 1), (1, 64)):
        tr = gpu_trace(w, launch=api.make_launch(tile, 2))
        _compare_forward(w, tr)


def test_forward_pixel_subsets_and_empty():
    w = unit_box_workload()
    rng = np.random.default_rng(3)
    ids = np.sort(rng.choice(64 * 64, 777, replace=False)).astype(np.int32)
    w.pixel_ids = ids
    tr = gpu_trace(w)
    _compare_forward(w, tr)
    w.pixel_ids = np.zeros(0, np.int32)
    tr = gpu_trace(w, render=True)
    assert tr.n_steps[0].numel() == 0


def test_forward_statuses_truncated_and_nonfinite():
    w = unit_box_workload(32, 32)
    w.scene = w.scene.replace(max_steps=7)
    tr = gpu_trace(w)
    _compare_forward(w, tr)
    assert (_np(tr.status[0]) & oracle.RAY_TRUNCATED).sum() > 0
    w = unit_box_workload(16, 16)
    w.T32 = w.T32.copy()
    w.T32[10:20, 10:20, 10:20] = np.nan
    tr = gpu_trace(w)
    _, ref = oracle_forward(w, stored_delta(w.T32))
    st = _np(tr.status[0])
    assert np.array_equal(st & oracle.RAY_NONFINITE, ref["status"] & oracle.RAY_NONFINITE)
    assert (st & oracle.RAY_NONFINITE).sum() > 0
    assert np.array_equal(_np(tr.n_steps[0]), ref["n_steps"])


def test_forward_persistent_equals_grid_bitwise():
    w = room_workload((64, 64, 48), 192, 160, seed=7)
    a = gpu_trace(w)
    b = gpu_trace(w, launch=api.make_launch((8, 8), 4, persistent=True, blocks_per_cu=2))
    for x, y in ((a.uv[0], b.uv[0]), (a.duv[0], b.duv[0]), (a.n_steps[0], b.n_steps[0]), (a.image[0], b.image[0])):
        assert torch.equal(x, y)


def test_forward_deterministic():
    w = room_workload((64, 64, 48), 128, 128, seed=8)
    a = gpu_trace(w)
    b = gpu_trace(w)
    assert torch.equal(a.uv[0], b.uv[0]) and torch.equal(a.n_steps[0], b.n_steps[0])
