"""Pins for the oracle's wall luminance (Sec. 2.C, Eq. 2 with one ray per pixel centre):
printed texture and pinhole projector, bilinear with zero padding."""

import numpy as np
import pytest

import oracle
from bos_inputs import scene_unit_box, scene_room


def _printed(pat):
    sc = scene_unit_box()
    return sc.replace(pat_h=pat.shape[0], pat_w=pat.shape[1])


def test_printed_texel_centres_return_texel_values():
    rng = np.random.default_rng(0)
    pat = rng.random((16, 24))
    sc = _printed(pat)
    Eu, Ev = sc.pat_extent_u, sc.pat_extent_v
    tu, tv = Eu / 24, Ev / 16
    rows, cols = np.meshgrid(np.arange(16), np.arange(24), indexing="ij")
    u = -Eu / 2 + (cols.ravel() + 0.5) * tu     # texture spans [-E/2, E/2], column 0 left
    v = Ev / 2 - (rows.ravel() + 0.5) * tv      # row 0 at the top
    img, _, st = oracle.render(sc, pat, np.stack([u, v], 1), np.zeros(u.size, np.uint8))
    assert np.allclose(img, pat.ravel(), atol=1e-12) and np.all(st == 0)


def test_printed_constant_and_affine_patterns():
    sc = _printed(np.zeros((32, 32)))
    rng = np.random.default_rng(1)
    inner = 0.8 * sc.pat_extent_u / 2
    uv = rng.uniform(-inner, inner, (500, 2))
    st = np.zeros(500, np.uint8)
    img, dI, _ = oracle.render(sc, np.full((32, 32), 0.37), uv, st)
    assert np.allclose(img, 0.37, atol=1e-14) and np.allclose(dI, 0.0, atol=1e-12)
    r, c = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    aff = 0.2 + 0.01 * c - 0.02 * r
    img, dI, _ = oracle.render(sc, aff, uv, st)
    # affine texture -> affine image with constant gradient in (u, v)
    assert np.allclose(dI, dI[0], atol=1e-10)
    pred = img[0] + (uv - uv[0]) @ dI[0]
    assert np.allclose(img, pred, atol=1e-12)


def test_printed_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    pat = rng.random((64, 64))
    sc = _printed(pat)
    tau = sc.pat_extent_u / 64
    uv = rng.uniform(-0.9, 0.9, (200, 2))
    a = (uv[:, 0] + sc.pat_extent_u / 2) / tau - 0.5
    b = (sc.pat_extent_v / 2 - uv[:, 1]) / tau - 0.5
    keep = (np.minimum(a % 1, 1 - a % 1) > 0.01) & (np.minimum(b % 1, 1 - b % 1) > 0.01)
    uv = uv[keep]
    st = np.zeros(len(uv), np.uint8)
    _, dI, _ = oracle.render(sc, pat, uv, st)
    e = 1e-6 * tau
    for k, off in enumerate(([e, 0.0], [0.0, e])):
        ip, _, _ = oracle.render(sc, pat, uv + off, st)
        im, _, _ = oracle.render(sc, pat, uv - np.array(off), st)
        assert np.allclose(dI[:, k], (ip - im) / (2 * e), rtol=1e-6, atol=1e-6)


def test_zero_padding_and_off_pattern_flag():
    pat = np.ones((8, 8))
    sc = _printed(pat)
    uv = np.array([[5.0, 5.0], [0.0, 0.0]])
    img, dI, st = oracle.render(sc, pat, uv, np.zeros(2, np.uint8))
    assert img[0] == 0.0 and st[0] & oracle.RAY_OFF_PATTERN
    assert img[1] == pytest.approx(1.0) and st[1] == 0


def test_projector_pixel_rays_land_on_their_texels():
    """Shooting a ray from the projector through texel centre (r, c) (same pinhole model as
    the camera) and rendering its wall point returns exactly that texel's value."""
    rng = np.random.default_rng(3)
    sc = scene_room((16, 16, 12), 8, 8, 64, pat=48)
    pat = rng.random((48, 48))
    proj_as_cam = sc.replace(cam_pos=sc.proj_pos, cam_fwd=sc.proj_fwd, cam_right=sc.proj_right,
                             cam_up=sc.proj_up, fov_x_deg=sc.proj_fov_x_deg, width=48, height=48)
    uv = []
    for pix in range(48 * 48):
        o, d = oracle.camera_ray(proj_as_cam, pix)
        s = (sc.wall_origin[1] - o[1]) / d[1]
        X = o + s * d
        uv.append([X[0] - sc.wall_origin[0], X[2] - sc.wall_origin[2]])
    img, _, st = oracle.render(sc, pat, np.array(uv), np.zeros(48 * 48, np.uint8))
    assert np.allclose(img, pat.ravel(), atol=1e-10) and np.all(st == 0)


def test_projector_axis_hits_image_centre_and_fd_gradient():
    rng = np.random.default_rng(4)
    sc = scene_room((16, 16, 12), 8, 8, 64, pat=64)
    pat = rng.random((64, 64))
    # the projector axis meets the wall at (proj x, proj z): image centre = mean of 4 texels
    uv_axis = np.array([[sc.proj_pos[0] - sc.wall_origin[0], sc.proj_pos[2] - sc.wall_origin[2]]])
    img, _, _ = oracle.render(sc, pat, uv_axis, np.zeros(1, np.uint8))
    assert img[0] == pytest.approx(pat[31:33, 31:33].mean(), abs=1e-13)
    uv = rng.uniform(-1.5, 1.5, (100, 2))
    st = np.zeros(100, np.uint8)
    _, dI, _ = oracle.render(sc, pat, uv, st)
    e = 1e-8
    for k, off in enumerate(([e, 0.0], [0.0, e])):
        ip, _, _ = oracle.render(sc, pat, uv + off, st)
        im, _, _ = oracle.render(sc, pat, uv - np.array(off), st)
        fd = (ip - im) / (2 * e)
        good = np.abs(fd - dI[:, k]) <= 1e-5 * (1 + np.abs(dI[:, k]))
        assert good.mean() > 0.95   # a few samples straddle a texel edge
