"""Pins for the oracle's field sampler (cell-centred trilinear interpolation, clamp to
edge, with the interpolant's exact gradient and Hessian).

Checked against SciPy's RegularGridInterpolator, exact reproduction of linear fields,
voxel-centre values and finite differences.
"""

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
from bos_inputs import voxel_centres

LO, HI, DIMS = (0.0, -0.5, 0.2), (1.0, 1.5, 1.1), (7, 9, 5)


def _field(rng):
    nx, ny, nz = DIMS
    return rng.standard_normal((nz, ny, nx))


def _interior_points(rng, n):
    xs, ys, zs = voxel_centres(LO, HI, DIMS)
    return np.stack([rng.uniform(c[0], c[-1], n) for c in (xs, ys, zs)], axis=1)


def test_matches_scipy_linear_interpolation():
    rng = np.random.default_rng(0)
    d = _field(rng)
    F = oracle.grid_field(d, LO, HI)
    xs, ys, zs = voxel_centres(LO, HI, DIMS)
    ref = RegularGridInterpolator((zs, ys, xs), d, method="linear")
    for P in _interior_points(rng, 300):
        val, _, _ = oracle.sample(F, P)
        assert val == pytest.approx(float(ref(P[::-1])[0]), abs=1e-13)


def test_voxel_centres_return_voxel_values():
    rng = np.random.default_rng(1)
    d = _field(rng)
    F = oracle.grid_field(d, LO, HI)
    xs, ys, zs = voxel_centres(LO, HI, DIMS)
    for _ in range(50):
        i, j, k = rng.integers(0, DIMS[0]), rng.integers(0, DIMS[1]), rng.integers(0, DIMS[2])
        val, _, _ = oracle.sample(F, (xs[i], ys[j], zs[k]))
        assert val == pytest.approx(d[k, j, i], abs=1e-14)


def test_linear_field_reproduced_exactly():
    rng = np.random.default_rng(2)
    g = np.array([0.3, -0.7, 1.1])
    xs, ys, zs = voxel_centres(LO, HI, DIMS)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    d = 0.25 + g[0] * X + g[1] * Y + g[2] * Z
    F = oracle.grid_field(d, LO, HI)
    for P in _interior_points(rng, 200):
        val, grad, hess = oracle.sample(F, P)
        assert val == pytest.approx(0.25 + g @ P, abs=1e-13)
        assert np.allclose(grad, g, atol=1e-12)
        assert np.allclose(hess, 0.0, atol=1e-11)


def test_gradient_and_hessian_are_derivatives_of_the_interpolant():
    rng = np.random.default_rng(3)
    d = _field(rng)
    F = oracle.grid_field(d, LO, HI)
    vox = (np.array(HI) - np.array(LO)) / np.array(DIMS)
    eps = 1e-6
    checked = 0
    for P in _interior_points(rng, 400):
        u = (P - np.array(LO)) / vox - 0.5
        frac = u - np.floor(u)
        if np.any(frac < 0.01) or np.any(frac > 0.99):
            continue  # keep the difference stencil inside one cell
        val, grad, hess = oracle.sample(F, P)
        for a in range(3):
            e = np.zeros(3)
            e[a] = eps
            vp, gp, _ = oracle.sample(F, P + e)
            vm, gm, _ = oracle.sample(F, P - e)
            assert grad[a] == pytest.approx((vp - vm) / (2 * eps), rel=1e-6, abs=1e-8)
            fd_h = (gp - gm) / (2 * eps)
            for b in range(3):
                if b != a:
                    assert hess[a, b] == pytest.approx(fd_h[b], rel=1e-5, abs=1e-6)
            assert hess[a, a] == 0.0  # trilinear: no pure second derivative within a cell
        checked += 1
    assert checked > 100


def test_clamp_to_edge_outside_centre_range():
    rng = np.random.default_rng(4)
    d = _field(rng)
    F = oracle.grid_field(d, LO, HI)
    xs, ys, zs = voxel_centres(LO, HI, DIMS)
    y, z = 0.5 * (ys[2] + ys[3]), 0.5 * (zs[1] + zs[2])
    inner, _, _ = oracle.sample(F, (xs[0], y, z))
    for x in (LO[0], 0.5 * (LO[0] + xs[0]), LO[0] - 0.3):
        val, grad, hess = oracle.sample(F, (x, y, z))
        assert val == pytest.approx(inner, abs=1e-14)
        assert grad[0] == 0.0 and hess[0, 1] == 0.0 and hess[0, 2] == 0.0
    outer, _, _ = oracle.sample(F, (xs[-1], y, z))
    val, grad, _ = oracle.sample(F, (HI[0] + 0.2, y, z))
    assert val == pytest.approx(outer, abs=1e-14) and grad[0] == 0.0


@pytest.mark.parametrize("mode,kw", [
    (oracle.oracle.FIELD_LINEAR, dict(a=2.7e-4, g=(1e-3, -2e-3, 5e-4), c=(0.5, 0.5, 0.5))),
    (oracle.oracle.FIELD_ETA2_LINEAR, dict(a=1.0006, g=(2e-3, 1e-3, -3e-3), c=(0.5, 0.5, 0.5))),
    (oracle.oracle.FIELD_GAUSSIAN, dict(a=2.7e-4, eps=-1e-5, c=(0.4, 0.6, 0.5), sigma=0.15)),
])
def test_analytic_field_derivatives(mode, kw):
    F = oracle.analytic_field(mode, (0, 0, 0), (1, 1, 1), **kw)
    rng = np.random.default_rng(5)
    eps = 1e-5
    for P in rng.uniform(0.1, 0.9, (20, 3)):
        val, grad, hess = oracle.sample(F, P)
        for a in range(3):
            e = np.zeros(3)
            e[a] = eps
            vp, gp, _ = oracle.sample(F, P + e)
            vm, gm, _ = oracle.sample(F, P - e)
            assert grad[a] == pytest.approx((vp - vm) / (2 * eps), rel=1e-6, abs=1e-12)
            assert np.allclose(hess[a], (gp - gm) / (2 * eps), rtol=1e-5, atol=1e-10)
        if mode == oracle.oracle.FIELD_ETA2_LINEAR:
            eta = 1.0 + val
            assert eta * eta == pytest.approx(kw["a"] + np.dot(kw["g"], P - np.array(kw["c"])), rel=1e-14)
