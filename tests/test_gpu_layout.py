"""The x-pair field layout (each voxel stored with its +x neighbour) against the cell
records: the stored codes bit for bit against the oracle's encoding, and the traced rays
and gradients of both layouts against each other and against the oracle. Both layouts hold
the same codes and the kernels do the same arithmetic on them, so exits, step counts and
statuses must be identical and gradients equal up to the order of the FP64 additions."""

import numpy as np
import pytest
import torch

import oracle
from _common import (CODES, RHO0G, T0, exit_error, expected_scale, grad_errors, oracle_forward, room_workload,
                     stored_delta, unit_box_workload)
from paper_2509_14442_amd import api
from test_gpu_forward import DEV, _np

pytestmark = pytest.mark.gpu


def _expected_pairs(codes: np.ndarray) -> np.ndarray:
    """X-pair entries (k, j, i), i in [-1, nx-1], j in [-1, ny], k in [-1, nz]: the codes of
    voxels (clamp(i), clamp(j), clamp(k)) and (clamp(i + 1), clamp(j), clamp(k))."""
    nz, ny, nx = codes.shape
    ix, iy, iz = np.arange(-1, nx), np.arange(-1, ny + 1), np.arange(-1, nz + 1)
    Y, Z = np.clip(iy, 0, ny - 1), np.clip(iz, 0, nz - 1)
    out = np.empty((nz + 2, ny + 2, nx + 1, 2), codes.dtype)
    for a in range(2):
        X = np.clip(ix + a, 0, nx - 1)
        out[..., a] = codes[Z][:, Y][:, :, X]
    return out


@pytest.mark.parametrize("dtype", ["f32-xpair", "f16-xpair", "bf16-xpair"])
def test_xpair_codes_bit_exact(dtype):
    w = room_workload((37, 23, 19), 8, 8, seed=5)
    field = api.Field.from_temperature(torch.from_numpy(w.T32).to(DEV), dtype)
    torch.cuda.synchronize()
    nx, ny, nz = field.dims
    f32 = dtype.startswith("f32")
    got = _np(field.buf).view(np.uint32 if f32 else np.uint16).reshape(nz + 2, ny + 2, nx + 1, 2)
    offset = 0.0 if f32 else RHO0G
    scale = expected_scale(w.T32, dtype, offset)
    assert field.scale == scale and field.offset == offset
    ref = oracle.encode(oracle.delta_from_temperature_f32(w.T32, RHO0G, T0), CODES[dtype], scale, offset)
    ref = ref.view(np.uint32) if f32 else ref
    assert np.array_equal(got, _expected_pairs(ref))


def _run(w, dtype, ckpt, launch=None, lam=None):
    field = api.Field.from_temperature(torch.from_numpy(w.T32).to(DEV), dtype)
    sc = api.Scene(w.scene, field, torch.from_numpy(w.pattern32).to(DEV), ckpt_stride=ckpt)
    tr = api.Tracer([sc], launch)
    tr.forward().render()
    g = tr.adjoint(dL_duv=[torch.from_numpy(lam).to(DEV)])[0] if lam is not None else None
    torch.cuda.synchronize()
    return tr, (None if g is None else _np(g)), field


@pytest.mark.parametrize("code,ckpt", [("f32", 3), ("f32", 6), ("bf16", 3), ("f16", 16)])
def test_xpair_equals_cell_records_and_oracle(code, ckpt):
    w = room_workload((40, 36, 28), 120, 88, seed=7, ckpt=ckpt, pat=256)
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((120 * 88, 2)).astype(np.float32)
    launch = api.make_launch((8, 8), 2, True, 0)
    tc, gc, fc = _run(w, code, ckpt, launch, lam)
    tx, gx, fx = _run(w, code + "-xpair", ckpt, launch, lam)
    assert fc.scale == fx.scale and fc.offset == fx.offset
    assert torch.equal(tc.uv[0], tx.uv[0]) and torch.equal(tc.n_steps[0], tx.n_steps[0])
    assert torch.equal(tc.status[0], tx.status[0]) and torch.equal(tc.image[0], tx.image[0])
    assert np.abs(gx - gc).max() <= 1e-12 * np.abs(gc).max()
    # and the oracle on the stored values
    delta = stored_delta(w.T32, code, fx.scale, fx.offset)
    F, ref = oracle_forward(w, delta)
    ok = np.isfinite(ref["uv"][:, 0])
    assert exit_error(_np(tx.uv[0])[ok], ref["uv"][ok]).max() <= 1e-6
    assert (_np(tx.n_steps[0]) != ref["n_steps"]).sum() <= 2
    g_ref = oracle.adjoint(F, w.scene, lam.astype(np.float64))
    l2, frac = grad_errors(gx, g_ref)
    assert l2 < 1e-3 and frac < 5e-3, (l2, frac)


def test_xpair_unit_box_edges():
    """Rays that cross the box faces sample the apron rows and planes of the pair array."""
    w = unit_box_workload(48, 48)
    rng = np.random.default_rng(9)
    lam = rng.standard_normal((48 * 48, 2)).astype(np.float32)
    tx, gx, _ = _run(w, "f32-xpair", 3, None, lam)
    F, ref = oracle_forward(w, stored_delta(w.T32))
    ok = np.isfinite(ref["uv"][:, 0])
    assert exit_error(_np(tx.uv[0])[ok], ref["uv"][ok]).max() <= 1e-6
    assert np.array_equal(_np(tx.n_steps[0]), ref["n_steps"])
    g_ref = oracle.adjoint(F, w.scene, lam.astype(np.float64))
    l2, frac = grad_errors(gx, g_ref)
    assert l2 < 1e-3 and frac < 2e-3, (l2, frac)
