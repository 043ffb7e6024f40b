"""Pins for the oracle's ray tracer: Eq. (1), dx/dt = v, dv/dt = eta grad(eta), integrated
with Sharma's Runge-Kutta-Nystrom scheme, plus the pinhole camera, box and wall.

Closed forms: straight rays in a homogeneous medium; cosh/sinh paths when eta is linear
in one direction; exact parabolas when eta^2 is linear. Convergence: fourth order in the
step on a smooth field, for the state, the invariant |v|^2 - eta^2 and reversibility.
Perturbation theory: the weak-field deflection integral of a Gaussian.
"""

import math

import numpy as np
import pytest

import oracle
from bos_inputs import scene_unit_box, scene_room, voxel_centres

F_GAUSS = oracle.oracle.FIELD_GAUSSIAN
F_ETA2 = oracle.oracle.FIELD_ETA2_LINEAR
F_HOMOG = oracle.oracle.FIELD_HOMOGENEOUS


# --- camera --------------------------------------------------------------------------------

def test_camera_centre_and_edges():
    sc = scene_unit_box().replace(width=65, height=33)
    o, d = oracle.camera_ray(sc, (33 // 2) * 65 + 65 // 2)
    assert np.allclose(o, sc.cam_pos) and np.allclose(d, sc.cam_fwd, atol=1e-15)
    # leftmost / rightmost pixel centres subtend the FOV less one pixel
    t = math.tan(math.radians(20.0))
    row = 16
    _, dl = oracle.camera_ray(sc, row * 65 + 0)
    _, dr = oracle.camera_ray(sc, row * 65 + 64)
    ang = math.acos(np.dot(dl, dr))
    assert ang == pytest.approx(2 * math.atan((1 - 1 / 65) * t), rel=1e-12)
    # row 0 is the top row, column 0 the left column
    _, d00 = oracle.camera_ray(sc, 0)
    assert np.dot(d00, sc.cam_up) > 0 and np.dot(d00, sc.cam_right) < 0
    assert np.linalg.norm(d00) == pytest.approx(1.0, abs=1e-15)


# --- homogeneous medium: straight rays -----------------------------------------------------

def test_homogeneous_medium_straight_rays():
    sc = scene_unit_box().replace(width=24, height=20)
    nx, ny, nz = sc.dims
    F = oracle.grid_field(np.full((nz, ny, nx), 2.7e-4), sc.box_lo, sc.box_hi)
    out = oracle.trace(F, sc)
    # analytic line-plane intersection from the camera
    for pix in range(sc.width * sc.height):
        o, d = oracle.camera_ray(sc, pix)
        s = (sc.wall_origin[1] - o[1]) / d[1]
        X = o + s * d
        u, v = X[0] - sc.wall_origin[0], X[2] - sc.wall_origin[2]
        assert out["uv"][pix, 0] == pytest.approx(u, abs=1e-12)
        assert out["uv"][pix, 1] == pytest.approx(v, abs=1e-12)
    assert np.abs(out["duv"]).max() < 1e-12
    entered = (out["status"] & oracle.RAY_MISSED_BOX) == 0
    assert entered.sum() > 0 and np.all(out["n_steps"][entered] >= 1)
    assert np.all(out["n_steps"][~entered] == 0)


# --- eta linear in one direction: cosh / sinh ------------------------------------------------

def _linear_grid(g, a, lo=(0, 0, 0), hi=(1, 1, 1), dims=(16, 16, 16)):
    xs, ys, zs = voxel_centres(lo, hi, dims)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return oracle.grid_field(a - 1.0 + g[0] * X + g[1] * Y + g[2] * Z, lo, hi)


def _linear_eta_closed_form(g, a, x0, v0, t):
    g = np.asarray(g, float)
    gam = np.linalg.norm(g)
    gh = g / gam
    w0 = a + g @ x0                     # eta(x0)
    c0 = gh @ v0
    w = w0 * math.cosh(gam * t) + c0 * math.sinh(gam * t)
    gv = w0 * math.sinh(gam * t) + c0 * math.cosh(gam * t)
    s = (w - a) / gam                   # gh . x(t), since eta = a + gam gh.x
    x_perp = (x0 - (gh @ x0) * gh) + (v0 - c0 * gh) * t
    v_perp = v0 - c0 * gh
    return x_perp + s * gh, v_perp + gv * gh


def test_linear_eta_cosh_sinh_and_fourth_order():
    g, a = (0.35, 0.1, -0.05), 1.2          # strong gradient so RK4 error is visible
    F = _linear_grid(g, a)
    x0 = np.array([0.25, 0.15, 0.5])
    d = np.array([0.25, 0.95, 0.05])
    d /= np.linalg.norm(d)
    v0 = (a + np.dot(g, x0)) * d
    t_end = 0.64
    xe, ve = _linear_eta_closed_form(g, a, x0, v0, t_end)
    errs = []
    for n in (8, 16, 32):
        x, v = oracle.integrate(F, x0, v0, t_end / n, n)
        errs.append(max(np.abs(x - xe).max(), np.abs(v - ve).max()))
    assert errs[-1] < 1e-7
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


# --- eta^2 linear: constant force, exact parabola ----------------------------------------------

def test_eta2_linear_exact_parabola_analytic():
    g = np.array([2e-2, -1e-2, 3e-2])
    F = oracle.analytic_field(F_ETA2, (0, 0, 0), (1, 1, 1), a=1.0006, g=g, c=(0.5, 0.5, 0.5))
    x0 = np.array([0.1, 0.0, 0.4])
    d = np.array([0.1, 1.0, 0.2])
    d /= np.linalg.norm(d)
    eta0 = math.sqrt(1.0006 + g @ (x0 - 0.5))
    v0 = eta0 * d
    for h, n in ((0.05, 20), (0.013, 77)):
        x, v = oracle.integrate(F, x0, v0, h, n)
        t = h * n
        assert np.allclose(x, x0 + v0 * t + g * t * t / 4, atol=1e-13, rtol=0)
        assert np.allclose(v, v0 + g * t / 2, atol=1e-13, rtol=0)


def test_eta2_linear_on_grid_close_to_parabola():
    # realistic magnitude: eta^2 - 1 ~ 5.4e-4 with a 1e-4 / m slope
    b = np.array([0.0, 0.0, 1e-4])
    a2 = (1 + 2.7e-4) ** 2
    lo, hi, dims = (0, 0, 0), (1, 1, 1), (32, 32, 32)
    xs, ys, zs = voxel_centres(lo, hi, dims)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    F = oracle.grid_field(np.sqrt(a2 + b[2] * (Z - 0.5)) - 1.0, lo, hi)
    x0 = np.array([0.5, 0.05, 0.5])
    eta0 = math.sqrt(a2)
    v0 = eta0 * np.array([0.0, 1.0, 0.0])
    h, n = 0.5 / 32, 56
    x, v = oracle.integrate(F, x0, v0, h, n)
    t = h * n
    assert np.abs(x - (x0 + v0 * t + b * t * t / 4)).max() < 1e-8


# --- fourth order on a smooth field, invariant, reversibility ---------------------------------

def _gauss():
    return oracle.analytic_field(F_GAUSS, (0, 0, 0), (1, 1, 1), a=0.3, eps=0.2, c=(0.55, 0.5, 0.45), sigma=0.2)


def _start():
    x0 = np.array([0.3, 0.05, 0.5])
    d = np.array([0.1, 1.0, -0.05])
    d /= np.linalg.norm(d)
    return x0, d


def test_rk4_fourth_order_gaussian():
    F = _gauss()
    x0, d = _start()
    eta0 = 1.0 + oracle.sample(F, x0)[0]
    v0 = eta0 * d
    T = 0.8
    xr, vr = oracle.integrate(F, x0, v0, T / 1024, 1024)
    errs = []
    for n in (16, 32, 64):
        x, v = oracle.integrate(F, x0, v0, T / n, n)
        errs.append(max(np.abs(x - xr).max(), np.abs(v - vr).max()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20, errs


def test_invariant_drift_fourth_order():
    # exact solutions keep |v|^2 = eta(x)^2 (Sharma's form of Eq. 1)
    F = _gauss()
    x0, d = _start()
    v0 = (1.0 + oracle.sample(F, x0)[0]) * d
    drift = []
    for n in (16, 32, 64):
        x, v = oracle.integrate(F, x0, v0, 0.8 / n, n)
        drift.append(abs(v @ v - (1.0 + oracle.sample(F, x)[0]) ** 2))
    # at least fourth order (the measured rate is about h^5 on this field)
    assert drift[0] / drift[1] > 12 and drift[1] / drift[2] > 12, drift


def test_reversibility_fourth_order():
    F = _gauss()
    x0, d = _start()
    v0 = (1.0 + oracle.sample(F, x0)[0]) * d
    errs = []
    for n in (16, 32, 64):
        h = 0.8 / n
        x, v = oracle.integrate(F, x0, v0, h, n)
        xb, vb = oracle.integrate(F, x, -v, h, n)
        errs.append(np.abs(xb - x0).max())
    # at least fourth order (about h^5 measured: the h^4 terms of the two legs largely cancel)
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12, errs


# --- weak-field deflection ---------------------------------------------------------------------

def test_weak_field_deflection_integral():
    """delta = delta0 + eps G(x), G a unit Gaussian of width sigma; a ray along +y at impact
    parameter b (in x) gains v_x = eps (-b sqrt(2 pi)/sigma) exp(-b^2/(2 sigma^2)) + O(eps^2)."""
    sigma, b, d0 = 0.1, 0.07, 2.7e-4
    rel = []
    for eps in (4e-4, 2e-4, 1e-4):
        F = oracle.analytic_field(F_GAUSS, (0, 0, 0), (1, 1, 1), a=d0, eps=eps, c=(0.5, 0.5, 0.5), sigma=sigma)
        x0 = np.array([0.5 + b, -0.5, 0.5])
        v0 = (1.0 + d0) * np.array([0.0, 1.0, 0.0])
        x, v = oracle.integrate(F, x0, v0, 0.002, 1000)
        pred = eps * (-b * math.sqrt(2 * math.pi) / sigma) * math.exp(-b * b / (2 * sigma * sigma))
        rel.append(abs(v[0] - pred) / abs(pred))
    assert rel[0] < 5e-3
    assert 1.6 < rel[0] / rel[1] < 2.5 and 1.6 < rel[1] / rel[2] < 2.5, rel


def test_rays_bend_away_from_hot_plume():
    # hot air is less dense: lower eta; rays bend toward higher eta, i.e. away from the plume
    from bos_inputs import fields

    sc = scene_unit_box().replace(width=1, height=1, fov_x_deg=1e-6)
    spec = fields.FieldSpec((fields.Plume((0.45, 0.5, 0.5), 8.0, 0.1),), 0.0)
    T = fields.temperature_grid(spec, sc.box_lo, sc.box_hi, sc.dims)
    F = oracle.grid_field(oracle.delta_from_temperature(T.astype(np.float32)), sc.box_lo, sc.box_hi)
    out = oracle.trace(F, sc)
    assert out["duv"][0, 0] > 1e-7   # plume at smaller x: the ray is pushed to larger u = x


# --- box statuses ---------------------------------------------------------------------------------

def test_box_statuses():
    sc = scene_unit_box().replace(width=16, height=16)
    nx, ny, nz = sc.dims
    d = np.full((nz, ny, nx), 2.7e-4)
    F = oracle.grid_field(d, sc.box_lo, sc.box_hi)
    # looking away from the box: every ray misses and goes straight
    away = sc.replace(cam_fwd=(0.0, -1.0, 0.0), cam_right=(-1.0, 0.0, 0.0),
                      wall_origin=(0.5, -3.0, 0.5), wall_normal=(0.0, 1.0, 0.0))
    out = oracle.trace(F, away)
    assert np.all(out["status"] == oracle.RAY_MISSED_BOX) and np.all(out["n_steps"] == 0)
    # too few steps: truncated, continues straight from the last state
    out = oracle.trace(F, sc.replace(max_steps=5))
    hit = (out["status"] & oracle.RAY_MISSED_BOX) == 0
    assert np.all(out["status"][hit] & oracle.RAY_TRUNCATED) and np.all(out["n_steps"][hit] == 5)
    # wall behind the camera: no wall hit
    out = oracle.trace(F, sc.replace(wall_normal=(0.0, 1.0, 0.0)))
    assert np.all(out["status"] & oracle.RAY_NO_WALL_HIT)
    # non-finite field values surface as NONFINITE rays
    d2 = d.copy()
    d2[:, :, :] = np.nan
    out = oracle.trace(oracle.grid_field(d2, sc.box_lo, sc.box_hi), sc)
    assert np.all(out["status"][hit] & oracle.RAY_NONFINITE) and np.all(out["n_steps"][hit] == 1)


def test_room_geometry_coverage():
    # the 40 degree camera at 5.5 m sees the full 4 m room width; projector covers all hits
    sc = scene_room((16, 16, 12), 64, 64, 512)
    nx, ny, nz = sc.dims
    F = oracle.grid_field(np.full((nz, ny, nx), 2.7e-4), sc.box_lo, sc.box_hi)
    out = oracle.trace(F, sc)
    assert np.all(out["status"] == 0)
    u = out["uv"][:, 0]
    assert u.min() > -2.05 and u.max() < 2.05 and u.max() - u.min() > 3.8
