"""Pins for the oracle's quasi-linear tracer (Sec. 2.B): the path is approximated by the
straight line L(t) = x0 + v0 t from the entry state, the field is queried on L to give
the velocity, and the velocity drives the position. The Sharma update is kept, with the
force taken on L at the stage times.

Closed forms and independent references:
  * homogeneous medium: straight rays, as in the nonlinear form;
  * eta^2 linear: the force is constant, so the quasi-linear path is the exact parabola;
  * the end state equals line integrals of the force along L, computed by adaptive
    quadrature of the sampled field: v = v0 + int D, x = x0 + v0 T + int (T - t) D,
    with the discretisation error falling as h^4;
  * weak fields: the velocity change is the first-order (Born) deflection integral;
  * the gap to the nonlinear path is second order in the field perturbation;
  * the gradient: dot-product identity with the tangent-linear model, and branch-locked
    central differences, including voxels of the entry layer (the line's direction
    v0 = (1 + delta(x0)) d depends on them).
"""

import math

import numpy as np
import pytest
from scipy import integrate as sint

import oracle
from bos_inputs import binary_dots, plume_unit_box, scene_unit_box, temperature_grid

F_GAUSS = oracle.oracle.FIELD_GAUSSIAN
F_ETA2 = oracle.oracle.FIELD_ETA2_LINEAR
QL = oracle.oracle.TRACER_QUASILINEAR


def test_homogeneous_medium_straight_rays_quasi():
    sc = scene_unit_box().replace(width=20, height=16, tracer=QL)
    nx, ny, nz = sc.dims
    F = oracle.grid_field(np.full((nz, ny, nx), 2.7e-4), sc.box_lo, sc.box_hi)
    out = oracle.trace(F, sc)
    for pix in range(sc.width * sc.height):
        o, d = oracle.camera_ray(sc, pix)
        s = (sc.wall_origin[1] - o[1]) / d[1]
        X = o + s * d
        assert out["uv"][pix, 0] == pytest.approx(X[0] - sc.wall_origin[0], abs=1e-12)
        assert out["uv"][pix, 1] == pytest.approx(X[2] - sc.wall_origin[2], abs=1e-12)
    assert np.abs(out["duv"]).max() < 1e-12


def test_eta2_linear_exact_parabola_quasi():
    """eta^2 = a + g.(x - c): D = eta grad(eta) = g / 2 everywhere, so the quasi-linear
    path is x0 + v0 t + g t^2 / 4 exactly."""
    g = np.array([0.02, -0.01, 0.03])
    F = oracle.analytic_field(F_ETA2, (0, 0, 0), (1, 1, 1), a=1.0005, g=tuple(g), c=(0.5, 0.5, 0.5))
    x0 = np.array([0.2, 0.1, 0.3])
    v0 = np.array([0.3, 0.9, 0.2])
    h, n = 0.01, 137
    x, v = oracle.integrate(F, x0, v0, h, n, quasi=True)
    t = h * n
    assert np.allclose(x, x0 + v0 * t + g * t * t / 4.0, rtol=0, atol=2e-14)
    assert np.allclose(v, v0 + g * t / 2.0, rtol=0, atol=2e-14)


def _line_integrals(F, x0, v0, T):
    """v0 + int_0^T D(L) dt and x0 + v0 T + int_0^T (T - t) D(L) dt by adaptive quadrature."""
    def D(t, a):
        d, grad, _ = oracle.sample(F, x0 + t * v0)
        return (1.0 + d) * grad[a]

    dv = np.array([sint.quad(D, 0.0, T, args=(a,), epsabs=1e-15, epsrel=1e-13, limit=200)[0] for a in range(3)])
    dx = np.array([sint.quad(lambda t, a: (T - t) * D(t, a), 0.0, T, args=(a,), epsabs=1e-15, epsrel=1e-13,
                             limit=200)[0] for a in range(3)])
    return x0 + v0 * T + dx, v0 + dv


def test_end_state_equals_line_integrals_fourth_order():
    F = oracle.analytic_field(F_GAUSS, (0, 0, 0), (1, 1, 1), a=2.7e-4, eps=3e-3, c=(0.48, 0.5, 0.55), sigma=0.12)
    x0 = np.array([0.52, 0.0, 0.47])
    v0 = (1.0 + 2.7e-4) * np.array([0.05, 0.99, -0.03]) / np.linalg.norm([0.05, 0.99, -0.03])
    T = 1.0
    x_ref, v_ref = _line_integrals(F, x0, v0, T)
    errs = []
    for n in (20, 40, 80):
        x, v = oracle.integrate(F, x0, v0, T / n, n, quasi=True)
        errs.append(max(np.abs(x - x_ref).max(), np.abs(v - v_ref).max()))
    assert errs[-1] < 1e-10, errs
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, (errs, r1, r2)


def test_weak_field_deflection_is_first_order_exact_quasi():
    """As for the nonlinear form: v_x = eps (-b sqrt(2 pi)/sigma) exp(-b^2/(2 sigma^2)) + O(eps^2)."""
    sigma, b, d0 = 0.1, 0.07, 2.7e-4
    rel = []
    for eps in (4e-4, 2e-4, 1e-4):
        F = oracle.analytic_field(F_GAUSS, (0, 0, 0), (1, 1, 1), a=d0, eps=eps, c=(0.5, 0.5, 0.5), sigma=sigma)
        x0 = np.array([0.5 + b, -0.5, 0.5])
        v0 = (1.0 + d0) * np.array([0.0, 1.0, 0.0])
        x, v = oracle.integrate(F, x0, v0, 0.002, 1000, quasi=True)
        pred = eps * (-b * math.sqrt(2 * math.pi) / sigma) * math.exp(-b * b / (2 * sigma * sigma))
        rel.append(abs(v[0] - pred) / abs(pred))
    assert rel[0] < 5e-3
    assert 1.6 < rel[0] / rel[1] < 2.5 and 1.6 < rel[1] / rel[2] < 2.5, rel


def test_gap_to_nonlinear_path_is_second_order():
    """Quasi-linear minus nonlinear end position scales as eps^2 (halving eps quarters it)."""
    sigma, b, d0 = 0.1, 0.05, 2.7e-4
    gaps, defl = [], []
    for eps in (2e-3, 1e-3, 5e-4):
        F = oracle.analytic_field(F_GAUSS, (0, 0, 0), (1, 1, 1), a=d0, eps=eps, c=(0.5, 0.5, 0.5), sigma=sigma)
        x0 = np.array([0.5 + b, -0.5, 0.5])
        v0 = (1.0 + d0) * np.array([0.0, 1.0, 0.0])
        xq, _ = oracle.integrate(F, x0, v0, 0.002, 1000, quasi=True)
        xn, _ = oracle.integrate(F, x0, v0, 0.002, 1000)
        gaps.append(np.linalg.norm(xq - xn))
        defl.append(abs(xn[0] - x0[0]))
    assert gaps[0] < 0.05 * defl[0]
    assert 3.5 < gaps[0] / gaps[1] < 4.5 and 3.5 < gaps[1] / gaps[2] < 4.5, gaps


def _setup(width, height, seed=1):
    sc = scene_unit_box().replace(width=width, height=height, tracer=QL)
    T = temperature_grid(plume_unit_box(seed), sc.box_lo, sc.box_hi, sc.dims)
    d = oracle.delta_from_temperature(T.astype(np.float32))
    return sc, oracle.grid_field(d, sc.box_lo, sc.box_hi), d


def test_dot_product_identity_quasi():
    sc, F, d = _setup(40, 36)
    rng = np.random.default_rng(17)
    v = rng.standard_normal(d.shape)
    w = rng.standard_normal((sc.width * sc.height, 2))
    lhs = float(np.sum(oracle.tangent(F, sc, v) * w))
    rhs = float(np.sum(v * oracle.adjoint(F, sc, w)))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs))
    assert abs(lhs) > 0


def test_quasi_adjoint_matches_locked_central_differences():
    sc, F, d = _setup(48, 48)
    pat = binary_dots(11)
    T2 = temperature_grid(plume_unit_box(2), sc.box_lo, sc.box_hi, sc.dims)
    F2 = oracle.grid_field(oracle.delta_from_temperature(T2.astype(np.float32)), sc.box_lo, sc.box_hi)
    fw2 = oracle.trace(F2, sc)
    target, _, _ = oracle.render(sc, pat, fw2["uv"], fw2["status"])
    fw = oracle.trace(F, sc)
    img, dI, _ = oracle.render(sc, pat, fw["uv"], fw["status"])
    _, dL = oracle.loss(img, target, dI)
    g = oracle.adjoint(F, sc, dL)
    rng = np.random.default_rng(19)
    gmax = np.abs(g).max()
    cand = np.flatnonzero(np.abs(g) > 1e-3 * gmax)
    # rays enter through the y = 0 face: voxels of the first layer also set the lines'
    # direction; include some of them explicitly
    nx, ny, nz = sc.dims
    j = (cand // nx) % ny
    entry = cand[j == 0]
    assert len(entry) >= 4
    vox = np.concatenate([rng.choice(cand, 16, replace=False), rng.choice(entry, 4, replace=False)])
    fd1 = oracle.fd_voxels(F, sc, pat, target, vox, h=1e-7, locked=True)
    fd2 = oracle.fd_voxels(F, sc, pat, target, vox, h=2e-7, locked=True)
    rich = (4.0 * fd1 - fd2) / 3.0
    ref = g.ravel()[vox]
    assert np.allclose(rich, ref, rtol=1e-6, atol=1e-9 * gmax), np.c_[rich, ref]


def test_quasi_gradient_zero_outside_ray_support_and_homogeneous():
    sc, F, d = _setup(1, 1)
    g = oracle.adjoint(F, sc, np.array([[1.0, -0.5]]))
    nz_idx = np.argwhere(g != 0.0)
    assert len(nz_idx) > 0
    assert set(nz_idx[:, 2]) <= {15, 16} and set(nz_idx[:, 0]) <= {15, 16}
    sc = scene_unit_box().replace(width=16, height=16, tracer=QL)
    nx, ny, nz = sc.dims
    Fh = oracle.grid_field(np.full((nz, ny, nx), 2.7e-4), sc.box_lo, sc.box_hi)
    fw = oracle.trace(Fh, sc)
    img, dI, _ = oracle.render(sc, np.full((256, 256), 0.5), fw["uv"], fw["status"])
    _, dL = oracle.loss(img, np.full(256, 0.1), dI)
    assert np.all(dL == 0.0) and np.all(oracle.adjoint(Fh, sc, dL) == 0.0)
