"""Pins for the oracle's pixel integral (Eq. 2): each pixel's value is the mean of spp
rays cast through sub-pixel points drawn from the triangular camera filter, each ray
carrying the wall radiance at its hit, optionally weighted by |<n_w, v_w>| / ell, ell the
length of the ray path (the polyline from the camera centre through the box entry and
every integrated state, then the signed straight continuation to the wall hit).

Independent references:
  * Philox-4x32-10 against the published known-answer vectors (tests/golden);
  * the sub-pixel offsets: the uniforms are the top 24 bits of the first two output
    words, and the offsets follow the triangular law (scipy's CDF, Kolmogorov-Smirnov,
    moments 0 and 1/6);
  * straight rays (homogeneous medium): projecting each hit point back onto the image
    plane gives the pixel centre plus that sample's offset, and the wall direction is
    the camera direction;
  * the radiometric weight of a straight ray is (n.d)^2 / D, D the camera-to-wall
    distance along the normal;
  * the path length: the camera-to-hit distance for straight rays; for eta^2 linear (the
    exact parabola) the polyline through the parabola's own points at the step times;
    never shorter than the chord, and longer by a second-order amount;
  * one sample per pixel and no weight is the centre-ray model, bit for bit;
  * the gradient including the direction term: dot-product identity with the
    tangent-linear model, and branch-locked central differences of the per-pixel loss.
"""

import math
from pathlib import Path

import ctypes as C
import numpy as np
import pytest
from scipy import stats

import oracle
from bos_inputs import binary_dots, plume_unit_box, scene_unit_box, temperature_grid

O = oracle.oracle
GOLDEN = Path(__file__).parent / "golden" / "philox4x32_10_kat.txt"
TENT = stats.triang(c=0.5, loc=-1.0, scale=2.0)


def test_philox_known_answers():
    rows = [ln.split() for ln in GOLDEN.read_text().splitlines() if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        w = [int(x, 16) for x in row]
        assert list(O.philox4x32(w[0:4], w[4:6])) == w[6:10]


def test_offsets_are_top_24_bits_through_the_tent_cdf():
    rng = np.random.default_rng(3)
    for _ in range(200):
        seed, pix, s = int(rng.integers(0, 2**32)), int(rng.integers(0, 2**31)), int(rng.integers(0, 1024))
        x = O.philox4x32([pix, s, 0, 0], [seed, 0])
        ox, oy = O.sample_offset(seed, pix, s)
        u = (x[:2] >> 8).astype(np.float64) * 2.0**-24
        assert abs(TENT.cdf(ox) - u[0]) < 1e-14 and abs(TENT.cdf(oy) - u[1]) < 1e-14
        assert -1.0 <= ox <= 1.0 and -1.0 <= oy <= 1.0


def test_offsets_follow_the_triangular_law():
    n = 40000
    off = np.array([O.sample_offset(7, p % 997, p // 997) for p in range(n)])
    for a in range(2):
        assert stats.kstest(off[:, a], TENT.cdf).pvalue > 1e-3
        assert abs(off[:, a].mean()) < 4.0 * math.sqrt(1.0 / 6.0 / n)
        assert abs(off[:, a].var() - 1.0 / 6.0) < 5e-3
    assert abs(np.corrcoef(off[:, 0], off[:, 1])[0, 1]) < 0.02
    # a different key gives different offsets, the same key the same ones
    assert O.sample_offset(8, 5, 1) != O.sample_offset(7, 5, 1)
    assert O.sample_offset(7, 5, 1) == O.sample_offset(7, 5, 1)


def _homogeneous(sc):
    nx, ny, nz = sc.dims
    return oracle.grid_field(np.full((nz, ny, nx), 2.7e-4), sc.box_lo, sc.box_hi)


def _pixel_coords(sc, X):
    """Project world points back to continuous pixel coordinates (col, row)."""
    c = np.asarray(sc.cam_pos)
    f, r, u = (np.asarray(a) for a in (sc.cam_fwd, sc.cam_right, sc.cam_up))
    rel = X - c
    z = rel @ f
    t = math.tan(math.radians(sc.fov_x_deg) / 2.0)
    px, py = (rel @ r) / z / t, (rel @ u) / z / t * sc.width / sc.height
    return (px + 1.0) * sc.width / 2.0, (1.0 - py) * sc.height / 2.0


def test_straight_rays_pass_through_offset_points():
    spp, seed = 5, 1234
    sc = scene_unit_box().replace(width=12, height=10, spp=spp, seed=seed)
    out = oracle.trace(_homogeneous(sc), sc)
    P = sc.width * sc.height
    O_w, eu, ev = (np.asarray(a) for a in (sc.wall_origin, sc.wall_u, sc.wall_v))
    X = O_w + out["uv"][:, :1] * eu + out["uv"][:, 1:] * ev
    col, row = _pixel_coords(sc, X)
    for r in range(P * spp):
        s, i = divmod(r, P)
        ox, oy = O.sample_offset(seed, i, s)
        assert col[r] == pytest.approx(i % sc.width + 0.5 + ox, abs=1e-9)
        assert row[r] == pytest.approx(i // sc.width + 0.5 + oy, abs=1e-9)
    d = (X - np.asarray(sc.cam_pos)) / np.linalg.norm(X - np.asarray(sc.cam_pos), axis=1, keepdims=True)
    assert np.abs(out["vdir"] - d).max() < 1e-12
    assert np.abs(out["duv"]).max() < 1e-12


def test_pixel_subset_reuses_the_pixels_own_samples():
    sc = scene_unit_box().replace(width=16, height=16, spp=3, seed=9)
    T = temperature_grid(plume_unit_box(1), sc.box_lo, sc.box_hi, sc.dims)
    F = oracle.grid_field(oracle.delta_from_temperature(T.astype(np.float32)), sc.box_lo, sc.box_hi)
    full = oracle.trace(F, sc)
    ids = np.array([3, 40, 41, 200, 255], np.int32)
    sub = oracle.trace(F, sc, ids)
    P = 256
    for s in range(3):
        assert np.array_equal(sub["uv"][s * len(ids):(s + 1) * len(ids)], full["uv"][s * P + ids])


def test_one_sample_no_weight_is_the_centre_model():
    sc = scene_unit_box().replace(width=20, height=18)
    T = temperature_grid(plume_unit_box(1), sc.box_lo, sc.box_hi, sc.dims)
    F = oracle.grid_field(oracle.delta_from_temperature(T.astype(np.float32)), sc.box_lo, sc.box_hi)
    fw = oracle.trace(F, sc)
    pat = binary_dots(4)
    img, dI, _ = oracle.render(sc, pat, fw["uv"], fw["status"])
    rp = oracle.render_pixels(sc, pat, fw["uv"], fw["status"])
    assert np.array_equal(img, rp["image"]) and np.array_equal(dI, rp["dI_duv"])
    assert not rp["dI_ddir"].any() and not rp["dI_dpath"].any()
    assert np.abs(np.linalg.norm(fw["vdir"], axis=1) - 1.0).max() < 1e-15
    # spp = 1 ignores the key: no offsets are drawn
    assert np.array_equal(oracle.trace(F, sc.replace(seed=99))["uv"], fw["uv"])


def test_pixel_value_is_the_mean_of_its_rays():
    spp = 6
    sc = scene_unit_box().replace(width=14, height=12, spp=spp, seed=77)
    T = temperature_grid(plume_unit_box(2), sc.box_lo, sc.box_hi, sc.dims)
    F = oracle.grid_field(oracle.delta_from_temperature(T.astype(np.float32)), sc.box_lo, sc.box_hi)
    fw = oracle.trace(F, sc)
    pat = binary_dots(5)
    img = oracle.render_pixels(sc, pat, fw["uv"], fw["status"])["image"]
    per_ray, _, _ = oracle.render(sc.replace(spp=1), pat, fw["uv"], fw["status"])
    P = sc.width * sc.height
    assert np.allclose(img, per_ray.reshape(spp, P).mean(0), rtol=0, atol=1e-15)


def test_radiometric_weight_of_straight_rays():
    spp = 4
    sc = scene_unit_box().replace(width=10, height=8, spp=spp, seed=5, radiometry=1)
    # a pattern wider than the view, so that no sample (offsets reach one pixel beyond
    # the pixel's edge) falls off it
    sc = sc.replace(pat_extent_u=1.5 * sc.pat_extent_u, pat_extent_v=1.5 * sc.pat_extent_v)
    fw = oracle.trace(_homogeneous(sc), sc)
    pat = np.full((sc.pat_h, sc.pat_w), 0.5)
    rp = oracle.render_pixels(sc, pat, fw["uv"], fw["status"], fw["vdir"], fw["path"])
    n = np.asarray(sc.wall_normal)
    D = abs(n @ (np.asarray(sc.wall_origin) - np.asarray(sc.cam_pos)))
    w = (fw["vdir"] @ n) ** 2 / D
    P = sc.width * sc.height
    assert np.allclose(rp["image"], 0.5 * w.reshape(spp, P).mean(0), rtol=1e-12, atol=0)
    assert not (rp["status"] & O.RAY_OFF_PATTERN).any()
    # straight rays: the path is the camera-to-hit distance
    X = np.asarray(sc.wall_origin) + fw["uv"][:, :1] * np.asarray(sc.wall_u) + fw["uv"][:, 1:] * np.asarray(sc.wall_v)
    assert np.allclose(fw["path"], np.linalg.norm(X - np.asarray(sc.cam_pos), axis=1), rtol=1e-13, atol=0)


def test_path_length_of_the_exact_parabola():
    """eta^2 = a + g.(x - c): the traced states are x0 + v0 t + g t^2 / 4 exactly, so the
    path is |x0 - cam| + the polyline through those points at t = 0, h, ..., N h + the
    straight segment to the wall."""
    g = np.array([0.004, 0.0, -0.006])
    sc = scene_unit_box().replace(width=5, height=4)
    F = oracle.analytic_field(O.FIELD_ETA2_LINEAR, sc.box_lo, sc.box_hi, a=1.0005, g=tuple(g), c=(0.5, 0.5, 0.5))
    out = oracle.trace(F, sc, want_exit=True)
    h = sc.step
    for pix in range(sc.width * sc.height):
        o, d = oracle.camera_ray(sc, pix)
        t_in = (sc.box_lo[1] - o[1]) / d[1]
        x0 = o + t_in * d
        eta0 = math.sqrt(1.0005 + g @ (x0 - np.array([0.5, 0.5, 0.5])))
        v0 = eta0 * d
        N = out["n_steps"][pix]
        t = h * np.arange(N + 1)
        pts = x0 + np.outer(t, v0) + np.outer(t * t, g) / 4.0
        xN, vN = out["exit_xv"][pix, :3], out["exit_xv"][pix, 3:]
        assert np.allclose(pts[-1], xN, atol=1e-12)
        s = ((np.asarray(sc.wall_origin) - xN) @ np.asarray(sc.wall_normal)) / (vN @ np.asarray(sc.wall_normal))
        ref = np.linalg.norm(x0 - o) + np.linalg.norm(np.diff(pts, axis=0), axis=1).sum() + s * np.linalg.norm(vN)
        assert out["path"][pix] == pytest.approx(ref, rel=1e-13)


def test_path_exceeds_the_chord_by_second_order():
    """In the room's plumes the path is never shorter than the camera-to-hit chord, and
    longer by far less than one FP32 ulp of it (the deflection angle is ~1e-5 rad)."""
    from bos_inputs import plumes_room, scene_room

    sc = scene_room((64, 64, 48), 96, 72)
    T = temperature_grid(plumes_room(3, sc.box_lo, sc.box_hi), sc.box_lo, sc.box_hi, sc.dims)
    F = oracle.grid_field(oracle.delta_from_temperature(T.astype(np.float32)), sc.box_lo, sc.box_hi)
    out = oracle.trace(F, sc)
    ok = np.isfinite(out["uv"][:, 0])
    X = (np.asarray(sc.wall_origin) + out["uv"][ok, :1] * np.asarray(sc.wall_u)
         + out["uv"][ok, 1:] * np.asarray(sc.wall_v))
    chord = np.linalg.norm(X - np.asarray(sc.cam_pos), axis=1)
    excess = (out["path"][ok] - chord) / chord
    assert excess.min() > -1e-14
    assert excess.max() < 1e-9, excess.max()


def _plume(sc, seed=1):
    T = temperature_grid(plume_unit_box(seed), sc.box_lo, sc.box_hi, sc.dims)
    d = oracle.delta_from_temperature(T.astype(np.float32))
    return oracle.grid_field(d, sc.box_lo, sc.box_hi), d


@pytest.mark.parametrize("tracer", [O.TRACER_NONLINEAR, O.TRACER_QUASILINEAR])
def test_dot_product_identity_with_direction_terms(tracer):
    sc = scene_unit_box().replace(width=24, height=20, spp=3, seed=11, radiometry=1, tracer=tracer)
    F, d = _plume(sc)
    ids = np.arange(0, 480, 2, dtype=np.int32)
    n = len(ids) * sc.spp
    rng = np.random.default_rng(17)
    v = rng.standard_normal(d.shape)
    w_uv, w_dir = rng.standard_normal((n, 2)), rng.standard_normal((n, 3))
    w_path = rng.standard_normal(n) * 1e3  # the path moves far less than the hit: scale up
    t_uv, t_dir, t_path = oracle.tangent(F, sc, v, ids, with_dir=True)
    lhs = float(np.sum(t_uv * w_uv) + np.sum(t_dir * w_dir) + np.sum(t_path * w_path))
    rhs = float(np.sum(v * oracle.adjoint(F, sc, w_uv, ids, dL_ddir=w_dir, dL_dpath=w_path)))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs))
    # the direction and path parts alone are non-trivial and satisfy it too
    z = np.zeros((n, 2))
    for wd, wp, t in ((w_dir, None, np.sum(t_dir * w_dir)), (None, w_path, np.sum(t_path * w_path))):
        r = float(np.sum(v * oracle.adjoint(F, sc, z, ids, dL_ddir=wd, dL_dpath=wp)))
        assert abs(r) > 1e-4 * abs(rhs)
        assert abs(t - r) <= 1e-10 * abs(r) + 1e-12 * abs(rhs)
    # and the direction stays unit: its tangent is orthogonal to it
    fw = oracle.trace(F, sc, ids)
    assert np.abs(np.sum(t_dir * fw["vdir"], axis=1)).max() <= 1e-12 * np.abs(t_dir).max()


@pytest.mark.parametrize("radiometry", [0, 1])
def test_pixel_loss_gradient_matches_locked_central_differences(radiometry):
    sc = scene_unit_box().replace(width=40, height=40, spp=4, seed=21, radiometry=radiometry)
    F, _ = _plume(sc, 1)
    F2, _ = _plume(sc, 2)
    pat = binary_dots(11)
    fw2 = oracle.trace(F2, sc)
    target = oracle.render_pixels(sc, pat, fw2["uv"], fw2["status"], fw2["vdir"], fw2["path"])["image"]
    fw = oracle.trace(F, sc)
    rp = oracle.render_pixels(sc, pat, fw["uv"], fw["status"], fw["vdir"], fw["path"])
    L, dL, dLd, dLp = oracle.loss_pixels(rp["image"], target, sc.spp, rp["dI_duv"],
                                         rp["dI_ddir"] if radiometry else None, rp["dI_dpath"] if radiometry else None)
    assert L > 0
    g = oracle.adjoint(F, sc, dL, dL_ddir=dLd, dL_dpath=dLp)
    gmax = np.abs(g).max()
    rng = np.random.default_rng(31)
    cand = np.flatnonzero(np.abs(g) > 1e-3 * gmax)
    vox = rng.choice(cand, 16, replace=False)
    fd1 = oracle.fd_voxels(F, sc, pat, target, vox, h=1e-7, locked=True)
    fd2 = oracle.fd_voxels(F, sc, pat, target, vox, h=2e-7, locked=True)
    rich = (4.0 * fd1 - fd2) / 3.0
    assert np.allclose(rich, g.ravel()[vox], rtol=1e-6, atol=1e-9 * gmax), np.c_[rich, g.ravel()[vox]]


def test_pixel_integral_argument_errors():
    sc = scene_unit_box().replace(width=4, height=4, spp=2)
    F = _homogeneous(sc)
    holder = oracle.oracle._SceneHolder(sc, None)
    uv = np.empty((5, 2))
    P = C.c_void_p
    rc = O.load().or_trace(F.ref, holder.ref, None, 5, uv.ctypes.data_as(P), None, None, None, None, None, None)
    assert rc < 0  # 5 rays is not a multiple of 2 samples per pixel
    rc = O.load().or_trace(F.ref, holder.ref, None, 16, uv.ctypes.data_as(P), None, None, None, None, None, None)
    assert rc < 0  # a full image needs width * height * spp rays
    with pytest.raises(Exception):
        oracle.trace(F, sc.replace(spp=0))
    pat = np.full((sc.pat_h, sc.pat_w), 0.5)
    fw = oracle.trace(F, sc.replace(radiometry=1))
    with pytest.raises(Exception):
        oracle.render_pixels(sc.replace(radiometry=1), pat, fw["uv"], fw["status"])  # weight needs vdir
    with pytest.raises(Exception):
        oracle.render_pixels(sc.replace(radiometry=1), pat, fw["uv"], fw["status"], fw["vdir"])  # and the path
