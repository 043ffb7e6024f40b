"""Pins for the oracle's gradient of L_BOS with respect to eta - 1 per voxel (Sec. 2.D,
computed by reverse mode through the discrete forward map).

The reverse mode is checked against an independently derived forward-mode
(tangent-linear) model through the dot-product identity <J v, w> = <v, J^T w>, and the
whole chain (trace, render, loss) against branch-locked central finite differences.
"""

import numpy as np
import pytest

import oracle
from bos_inputs import binary_dots, plume_unit_box, scene_unit_box, temperature_grid


def _setup(width=64, height=64, seed=1):
    sc = scene_unit_box().replace(width=width, height=height)
    T = temperature_grid(plume_unit_box(seed), sc.box_lo, sc.box_hi, sc.dims)
    d = oracle.delta_from_temperature(T.astype(np.float32))
    return sc, oracle.grid_field(d, sc.box_lo, sc.box_hi), d


def _loss_parts(F, sc, pat, target, ids=None):
    fw = oracle.trace(F, sc, ids)
    img, dI, st = oracle.render(sc, pat, fw["uv"], fw["status"])
    L, dL = oracle.loss(img, target, dI)
    return L, dL, img


def test_dot_product_identity_adjoint_vs_tangent():
    sc, F, d = _setup(48, 40)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(d.shape)
    w = rng.standard_normal((sc.width * sc.height, 2))
    Jv = oracle.tangent(F, sc, v)
    JTw = oracle.adjoint(F, sc, w)
    lhs = float(np.sum(Jv * w))
    rhs = float(np.sum(v * JTw))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs))
    assert abs(lhs) > 0


def test_adjoint_matches_locked_central_differences():
    sc, F, d = _setup(64, 64)
    pat = binary_dots(11)
    # target: the image of a second plume field
    T2 = temperature_grid(plume_unit_box(2), sc.box_lo, sc.box_hi, sc.dims)
    F2 = oracle.grid_field(oracle.delta_from_temperature(T2.astype(np.float32)), sc.box_lo, sc.box_hi)
    _, _, target = _loss_parts(F2, sc, pat, np.zeros(sc.width * sc.height))
    L, dL, _ = _loss_parts(F, sc, pat, target)
    g = oracle.adjoint(F, sc, dL)
    rng = np.random.default_rng(13)
    nx, ny, nz = sc.dims
    cand = np.flatnonzero(np.abs(g) > 1e-3 * np.abs(g).max())
    vox = rng.choice(cand, 24, replace=False)
    fd1 = oracle.fd_voxels(F, sc, pat, target, vox, h=1e-7, locked=True)
    fd2 = oracle.fd_voxels(F, sc, pat, target, vox, h=2e-7, locked=True)
    ref = g.ravel()[vox]
    # central differences carry an h^2 L'''/6 term that is not small relative to L' on rays
    # whose residual I - I* is near zero; Richardson extrapolation removes it
    rich = (4.0 * fd1 - fd2) / 3.0
    assert np.allclose(rich, ref, rtol=1e-6, atol=1e-9 * np.abs(g).max()), np.c_[rich, ref]
    assert np.allclose(fd1, ref, rtol=1e-4, atol=1e-9 * np.abs(g).max())
    # unlocked differences are close but may see branch jumps (diagnostic only)
    fdu = oracle.fd_voxels(F, sc, pat, target, vox[:6], h=1e-7, locked=False)
    assert np.allclose(fdu, ref[:6], rtol=0.2, atol=1e-3 * np.abs(g).max())


def test_gradient_zero_outside_ray_support():
    # a single ray along the box's central line touches only voxels with x, z index 15 or 16
    sc, F, d = _setup(1, 1)
    g = oracle.adjoint(F, sc, np.array([[1.0, -0.5]]))
    nz_idx = np.argwhere(g != 0.0)
    assert len(nz_idx) > 0
    assert set(nz_idx[:, 2]) <= {15, 16} and set(nz_idx[:, 0]) <= {15, 16}


def test_homogeneous_field_constant_pattern_zero_gradient():
    sc = scene_unit_box().replace(width=16, height=16)
    nx, ny, nz = sc.dims
    F = oracle.grid_field(np.full((nz, ny, nx), 2.7e-4), sc.box_lo, sc.box_hi)
    pat = np.full((256, 256), 0.5)
    L, dL, img = _loss_parts(F, sc, pat, np.full(256, 0.1))
    assert np.all(dL == 0.0)
    assert np.all(oracle.adjoint(F, sc, dL) == 0.0)


def test_pixel_subset_gradient_equals_restricted_full_gradient():
    sc, F, d = _setup(32, 32)
    rng = np.random.default_rng(9)
    w = rng.standard_normal((32 * 32, 2))
    ids = np.sort(rng.choice(32 * 32, 100, replace=False)).astype(np.int32)
    wm = np.zeros_like(w)
    wm[ids] = w[ids]
    g_full = oracle.adjoint(F, sc, wm)
    g_sub = oracle.adjoint(F, sc, w[ids], pixel_ids=ids)
    assert np.allclose(g_full, g_sub, rtol=1e-12, atol=1e-15 * np.abs(g_full).max())
