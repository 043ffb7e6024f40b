"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every entry
point that include/rbos.h declares, the binding's struct layouts match the compiled ones,
and invalid arguments are rejected before anything is enqueued."""

import ctypes as C
import os
import re

import pytest

import paper_2509_14442_amd._lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        import paper_2509_14442_amd.build as b

        b.build()
    return L.load()


def test_exports_match_header(lib):
    with open(os.path.join(ROOT, "include", "rbos.h")) as f:
        hdr = f.read()
    declared = set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(rbos_\w+)\s*\(", hdr, re.M))
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.rbos_version() == int(re.search(r"#define RBOS_ABI_VERSION (\d+)", hdr).group(1)) == 2


def test_struct_layouts_match(lib):
    for which, st in enumerate(L.STRUCTS):
        offs = (C.c_size_t * 64)()
        size = lib.rbos_struct_layout(which, offs, 64)
        assert size == C.sizeof(st), st.__name__
        for i, (name, _) in enumerate(st._fields_):
            assert offs[i] == getattr(st, name).offset, (st.__name__, name)
    assert lib.rbos_struct_layout(99, None, 0) == 0


def test_field_bytes(lib):
    # one record per cell of the padded grid (one apron cell on each side)
    assert lib.rbos_field_bytes(128, 128, 128, L.RBOS_F32) == 32 * 129 ** 3
    assert lib.rbos_field_bytes(128, 128, 128, L.RBOS_F16) == 16 * 129 ** 3
    assert lib.rbos_field_bytes(1, 4, 4, 0) == 0 and lib.rbos_field_bytes(449, 4, 4, 0) == 0
    assert lib.rbos_field_bytes(4, 4, 4, 7) == 0


def _valid_scene():
    s = L.rbos_scene()
    s.nx = s.ny = s.nz = 8
    s.box_lo, s.box_hi = L.D3(0, 0, 0), L.D3(1, 1, 1)
    s.dtype, s.enc_scale, s.enc_offset = 0, 1.0, 0.0
    s.field = 0x1000
    s.cam_pos, s.cam_fwd = L.D3(0.5, -1.5, 0.5), L.D3(0, 1, 0)
    s.cam_right, s.cam_up = L.D3(1, 0, 0), L.D3(0, 0, 1)
    s.cam_fov_x_deg = 40.0
    s.width = s.height = 4
    s.n_pixels = 16
    s.spp = 1
    s.wall_origin, s.wall_normal = L.D3(0.5, 1.5, 0.5), L.D3(0, -1, 0)
    s.wall_u, s.wall_v = L.D3(1, 0, 0), L.D3(0, 0, 1)
    s.wall_mode = 0
    s.pattern, s.pat_w, s.pat_h = 0x2000, 4, 4
    s.pat_extent_u = s.pat_extent_v = 1.0
    s.step, s.max_steps, s.ckpt_stride = 1 / 16, 64, 16
    return s


def _fwd(lib, s, outs=None, launch=None, ws=0x100000, ws_bytes=1 << 20):
    if outs is None:
        outs = L.rbos_trace_out(0x3000, 0x4000, 0x5000, 0x6000, 0x7000)
    rc = lib.rbos_trace_forward(C.byref(s), 1, C.byref(outs), C.byref(launch) if launch else None,
                                C.c_void_p(ws), ws_bytes, None)
    return rc, lib.rbos_last_error().decode()


@pytest.mark.parametrize("mutate,code", [
    (lambda s: setattr(s, "nx", 1), -2),
    (lambda s: setattr(s, "nz", 500), -2),
    (lambda s: setattr(s, "box_hi", L.D3(0, 1, 1)), -3),
    (lambda s: setattr(s, "dtype", 6), -4),
    (lambda s: setattr(s, "enc_scale", 3.0), -3),
    (lambda s: setattr(s, "field", None), -1),
    (lambda s: setattr(s, "cam_fwd", L.D3(0, 1, 0.1)), -3),
    (lambda s: setattr(s, "cam_fov_x_deg", 0.0), -3),
    (lambda s: setattr(s, "n_pixels", 15), -2),
    (lambda s: setattr(s, "spp", 0), -3),
    (lambda s: setattr(s, "spp", 1025), -3),
    (lambda s: setattr(s, "radiometry", 2), -3),
    (lambda s: setattr(s, "wall_normal", L.D3(0, -2, 0)), -3),
    (lambda s: setattr(s, "step", -1.0), -3),
    (lambda s: setattr(s, "step", 1.0), -3),
    (lambda s: setattr(s, "max_steps", 0), -3),
    (lambda s: setattr(s, "ckpt_stride", 12), -7),
    (lambda s: setattr(s, "ckpt_stride", 5), -7),
    (lambda s: setattr(s, "tracer", 2), -3),
    (lambda s: setattr(s, "ckpt_stride", 264), -7),
])
def test_forward_validation(lib, mutate, code):
    s = _valid_scene()
    mutate(s)
    rc, msg = _fwd(lib, s)
    assert rc == code, msg
    assert msg


def test_forward_output_and_workspace_checks(lib):
    s = _valid_scene()
    rc, msg = _fwd(lib, s, outs=L.rbos_trace_out(0, 0x4000, 0x5000, 0x6000, 0x7000))
    assert rc == -1 and "wall_uv" in msg
    rc, msg = _fwd(lib, s, outs=L.rbos_trace_out(0x3000, 0x4000, 0x5000, 0x6000, 0))
    assert rc == -1 and "ckpt" in msg
    for k in (1, 3, 4, 6, 8, 256):  # accepted strides: the error is the missing checkpoint buffer
        s.ckpt_stride = k
        rc, msg = _fwd(lib, s, outs=L.rbos_trace_out(0x3000, 0x4000, 0x5000, 0x6000, 0))
        assert rc == -1 and "ckpt" in msg, (k, msg)
    s.ckpt_stride = 16
    rc, msg = _fwd(lib, s, ws=0)
    assert rc == -5
    rc, msg = _fwd(lib, s, ws_bytes=16)
    assert rc == -5
    rc, msg = _fwd(lib, s, ws=0x100010)
    assert rc == -5 and "aligned" in msg
    bad = L.rbos_launch(8, 4, 4, 0, 1)
    rc, msg = _fwd(lib, s, launch=bad)
    assert rc == -3
    bad = L.rbos_launch(8, 8, 3, 0, 1)
    rc, msg = _fwd(lib, s, launch=bad)
    assert rc == -3


def test_render_and_adjoint_validation(lib):
    s = _valid_scene()
    outs = L.rbos_trace_out(0x3000, 0x4000, 0x5000, 0x6000, 0x7000)
    io = L.rbos_render_io(None, 0x8000, 0x9000, None)
    rc = lib.rbos_render(C.byref(s), 1, C.byref(outs), C.byref(io), C.c_void_p(0x100000), 1 << 20, None)
    assert rc == -1 and b"target" in lib.rbos_last_error()
    s.pattern = None
    io = L.rbos_render_io(None, 0x8000, None, None)
    rc = lib.rbos_render(C.byref(s), 1, C.byref(outs), C.byref(io), C.c_void_p(0x100000), 1 << 20, None)
    assert rc == -1 and b"pattern" in lib.rbos_last_error()
    # the radiometric weight needs the forward's wall directions, and its gradient a
    # direction seed per ray
    s = _valid_scene()
    s.radiometry = 1
    io = L.rbos_render_io(0x8800, 0x8000, None, None)
    rc = lib.rbos_render(C.byref(s), 1, C.byref(outs), C.byref(io), C.c_void_p(0x100000), 1 << 20, None)
    assert rc == -1 and b"wall_dir" in lib.rbos_last_error()
    outs_d = L.rbos_trace_out(0x3000, 0x4000, 0x5000, 0x6000, 0x7000, 0x7800)
    io = L.rbos_render_io(0x8800, 0x8000, 0x9000, None)
    rc = lib.rbos_render(C.byref(s), 1, C.byref(outs_d), C.byref(io), C.c_void_p(0x100000), 1 << 20, None)
    assert rc == -1 and b"dL_ddir" in lib.rbos_last_error()
    io = L.rbos_render_io(None, 0x8000, None, None, 0x9800)
    rc = lib.rbos_render(C.byref(s), 1, C.byref(outs_d), C.byref(io), C.c_void_p(0x100000), 1 << 20, None)
    assert rc == -1 and b"target" in lib.rbos_last_error()
    s = _valid_scene()
    s.ckpt_stride = 0
    aio = L.rbos_adjoint_io(0xa000, 0xb000)
    rc = lib.rbos_trace_adjoint(C.byref(s), 1, C.byref(outs), C.byref(aio), None, C.c_void_p(0x100000),
                                1 << 20, None)
    assert rc == -7
    s.ckpt_stride = 16
    aio = L.rbos_adjoint_io(0xa000, None)
    rc = lib.rbos_trace_adjoint(C.byref(s), 1, C.byref(outs), C.byref(aio), None, C.c_void_p(0x100000),
                                1 << 20, None)
    assert rc == -1


def test_field_validation_and_sizes(lib):
    assert lib.rbos_field_from_temperature(1, 4, 4, C.c_void_p(0x10), 2.7e-4, 293.0, 0, 1.0, 0.0,
                                           C.c_void_p(0x20), None) == -2
    assert lib.rbos_field_from_temperature(4, 4, 4, None, 2.7e-4, 293.0, 0, 1.0, 0.0, C.c_void_p(0x20), None) == -1
    assert lib.rbos_field_from_temperature(4, 4, 4, C.c_void_p(0x10), -1.0, 293.0, 0, 1.0, 0.0,
                                           C.c_void_p(0x20), None) == -3
    assert lib.rbos_field_encode(4, 4, 4, C.c_void_p(0x10), 7, 1.0, 0.0, C.c_void_p(0x20), None) == -4
    s = _valid_scene()
    # a 19-float ray header plus 6 floats per checkpoint slot, per entry: the image in
    # 8 x 8 pixel blocks (4 x 4 pixels: one block of 64 entries)
    assert (s.width, s.height, s.pixel_ids) == (4, 4, None)
    assert lib.rbos_ckpt_bytes(C.byref(s)) == (19 + ((64 - 1) // 16) * 6) * 64 * 4
    s.ckpt_stride = 1  # every step's state
    assert lib.rbos_ckpt_bytes(C.byref(s)) == (19 + (64 - 1) * 6) * 64 * 4
    s.width, s.height, s.n_pixels = 17, 9, 17 * 9  # 3 x 2 blocks
    assert lib.rbos_ckpt_bytes(C.byref(s)) == (19 + (64 - 1) * 6) * 6 * 64 * 4
    s.spp = 3  # one image plane per sample
    assert lib.rbos_ckpt_bytes(C.byref(s)) == (19 + (64 - 1) * 6) * 3 * 6 * 64 * 4
    s.pixel_ids, s.n_pixels = 0x40, 65  # pixel list: 65 x 3 rays -> 256 entries
    assert lib.rbos_ckpt_bytes(C.byref(s)) == (19 + (64 - 1) * 6) * 256 * 4
    s.spp = 1  # 65 rays -> 128 entries
    assert lib.rbos_ckpt_bytes(C.byref(s)) == (19 + (64 - 1) * 6) * 128 * 4
    s.tracer = L.RBOS_TRACER_QUASILINEAR  # the quasi-linear adjoint needs only the ray header
    assert lib.rbos_ckpt_bytes(C.byref(s)) == 19 * 128 * 4
    s.tracer = L.RBOS_TRACER_NONLINEAR
    s.ckpt_stride = 0
    assert lib.rbos_ckpt_bytes(C.byref(s)) == 0
    assert lib.rbos_workspace_bytes(C.byref(s), 1) >= 256
    # empty batch is a no-op
    assert lib.rbos_trace_forward(C.byref(s), 0, None, None, None, 0, None) == 0


def test_mlp_entry_point_validation(lib):
    assert lib.rbos_mlp_param_count(64, 4) == 3 * 64 + 64 + 3 * (64 * 64 + 64) + 64 * 5 + 5
    assert lib.rbos_mlp_param_count(32, 4) == 0 and lib.rbos_mlp_param_count(64, 0) == 0
    assert lib.rbos_mlp_param_count(64, 9) == 0
    n = 1000
    nb = lib.rbos_mlp_workspace_bytes(64, 4, n)
    assert nb >= 4 * n * 64 * 4 + 2 * n * 64 * 4
    m = L.rbos_mlp(64, 4, 0x1000, L.D3(0, 0, 0), L.D3(4, 4, 3))
    ws = C.c_void_p(0x100000)

    def fwd(mm, pts=0x2000, n=n, grid=None, ws=ws, nbytes=nb):
        rc = lib.rbos_mlp_forward(C.byref(mm) if mm is not None else None, C.c_void_p(pts) if pts else None, n,
                                  grid, C.c_void_p(0x3000), None, 0.0, 0.0, ws, nbytes, None)
        return rc, lib.rbos_last_error().decode()

    assert fwd(None)[0] == -1
    assert fwd(L.rbos_mlp(32, 4, 0x1000, L.D3(0, 0, 0), L.D3(4, 4, 3)))[0] == -7
    assert fwd(L.rbos_mlp(64, 4, None, L.D3(0, 0, 0), L.D3(4, 4, 3)))[0] == -1
    assert fwd(L.rbos_mlp(64, 4, 0x1000, L.D3(0, 0, 0), L.D3(4, 0, 3)))[0] == -3
    assert fwd(m, pts=0)[0] == -1  # neither points nor a grid
    assert fwd(m, pts=0, grid=(C.c_int32 * 3)(10, 10, 11))[0] == -2  # 1100 != 1000 points
    assert fwd(m, ws=None)[0] == -5
    assert fwd(m, nbytes=nb - 1)[0] == -5
    assert fwd(m, ws=C.c_void_p(0x100010))[0] == -5
    assert fwd(m, n=0, ws=None, nbytes=0)[0] == 0  # empty: nothing enqueued
    rc = lib.rbos_mlp_backward(C.byref(m), C.c_void_p(0x2000), n, None, C.c_void_p(0x3000), None, ws, nb, None)
    assert rc == -1 and b"dparams" in lib.rbos_last_error()
    assert lib.rbos_mlp_bos_seed(10, C.c_void_p(0x10), C.c_void_p(0x20), -1.0, 293.0, 303.0, C.c_void_p(0x30),
                                 None) == -3
    assert lib.rbos_mlp_bos_seed(10, None, C.c_void_p(0x20), 2.7e-4, 293.0, 303.0, C.c_void_p(0x30), None) == -1
    assert lib.rbos_mlp_bos_seed(0, None, None, 2.7e-4, 293.0, 303.0, None, None) == 0


def test_pde_and_fit_validation(lib):
    m = L.rbos_mlp(64, 3, 0x1000, L.D3(0, 0, 0), L.D3(1, 1, 1))
    pde = L.rbos_pde(50.0, 35.0, 0.8, 0.5, L.D3(1, 1, 1))
    nb = lib.rbos_mlp_pde_workspace_bytes(64, 3, 100)
    assert nb > 7 * 100 * 64 * 4 * 3
    ws = C.c_void_p(0x100000)

    def call(mm=m, pp=pde, pts=0x2000, n=100, w=ws, nbytes=nb):
        return lib.rbos_mlp_pde_loss(C.byref(mm), C.byref(pp) if pp is not None else None,
                                     C.c_void_p(pts) if pts else None, n, C.c_void_p(0x3000), None, None, w, nbytes,
                                     None)

    assert call(pp=None) == -1
    assert call(pts=0) == -1
    assert call(pp=L.rbos_pde(0.0, 35.0, 0.8, 0.5, L.D3(1, 1, 1))) == -3
    assert call(pp=L.rbos_pde(50.0, 35.0, 0.8, 0.5, L.D3(1, -1, 1))) == -3
    assert call(nbytes=nb - 1) == -5
    assert call(mm=L.rbos_mlp(64, 9, 0x1000, L.D3(0, 0, 0), L.D3(1, 1, 1))) == -7
    nrm = (C.c_double * 5)(1, 1, 1, 1, 0)
    assert lib.rbos_mlp_fit_seed(10, C.c_void_p(0x10), C.c_void_p(0x20), nrm, C.c_void_p(0x30), None, None, 0,
                                 None) == -3
    nrm = (C.c_double * 5)(1, 1, 1, 1, 1)
    assert lib.rbos_mlp_fit_seed(10, C.c_void_p(0x10), C.c_void_p(0x20), nrm, C.c_void_p(0x30), C.c_void_p(0x40),
                                 None, 0, None) == -5


def test_adjoint_noalloc_validation(lib):
    """The no-allocation adjoint checks its arguments like rbos_trace_adjoint, and rejects
    scenes whose scratch exceeds the static device array, all before any device call."""
    outs = L.rbos_trace_out(0x3000, 0x4000, 0x5000, 0x6000, 0x7000)
    aio = L.rbos_adjoint_io(0xa000, 0xb000)
    s = _valid_scene()
    s.ckpt_stride = 0
    assert lib.rbos_trace_adjoint_noalloc(C.byref(s), 1, C.byref(outs), C.byref(aio), None, None) == -7
    s.ckpt_stride = 16
    bad = L.rbos_adjoint_io(0xa000, None)
    assert lib.rbos_trace_adjoint_noalloc(C.byref(s), 1, C.byref(outs), C.byref(bad), None, None) == -1
    # 2048 x 2048 pixels x 64 samples: 4M tiles, 8 B of step count and order each
    s.width = s.height = 2048
    s.n_pixels = 2048 * 2048
    s.spp = 64
    rc = lib.rbos_trace_adjoint_noalloc(C.byref(s), 1, C.byref(outs), C.byref(aio), None, None)
    msg = lib.rbos_last_error().decode()
    assert rc == -5 and "static buffer" in msg and str(L.NOALLOC_SCRATCH_BYTES) in msg, msg
    # nothing to do: no device call either
    assert lib.rbos_trace_adjoint_noalloc(C.byref(s), 0, C.byref(outs), C.byref(aio), None, None) == 0


def test_code_scale(lib):
    """The library's 16-bit code scale: the largest power of two s with
    s * max |eta - 1 - c| <= 2^14, here checked against the tests' own derivation from the
    temperature range, and at the edges of its definition."""
    import numpy as np

    from _common import RHO0G, T0, expected_scale

    rng = np.random.default_rng(7)
    for _ in range(20):
        T = rng.uniform(280.0, 330.0, 64).astype(np.float32)
        for dtype, code in (("f16", L.RBOS_F16), ("bf16", L.RBOS_BF16), ("f32", L.RBOS_F32)):
            for c in (0.0, RHO0G):
                s = lib.rbos_code_scale_temperature(code, float(T.min()), float(T.max()), RHO0G, T0, c)
                assert s == expected_scale(T, dtype, c), (dtype, c, s)
    # a range whose largest |delta - c| is exactly 2^-16: s = 2^30 puts it at 2^14
    assert lib.rbos_code_scale(L.RBOS_F16, -2.0 ** -16, 2.0 ** -17, 0.0) == 2.0 ** 30
    assert lib.rbos_code_scale(L.RBOS_BF16, 1e-4, 1e-4, 1e-4) == 1.0  # nothing to store
    assert lib.rbos_code_scale(L.RBOS_F32, 0.0, 1.0, 0.5) == 1.0
    assert lib.rbos_code_scale(7, 0.0, 1.0, 0.0) == 0.0
    assert lib.rbos_code_scale(L.RBOS_F16, 1.0, 0.0, 0.0) == 0.0
    assert lib.rbos_code_scale_temperature(L.RBOS_F16, 0.0, 300.0, RHO0G, T0, 0.0) == 0.0


def test_field_bytes_xpair(lib):
    # x-pairs: (nx+1)(ny+2)(nz+2) entries of 8 B (FP32) or 4 B (two 16-bit codes)
    assert lib.rbos_field_bytes(128, 128, 128, L.RBOS_F32_XPAIR) == 8 * 129 * 130 * 130
    assert lib.rbos_field_bytes(256, 256, 192, L.RBOS_BF16_XPAIR) == 4 * 257 * 258 * 194
    assert lib.rbos_field_bytes(448, 448, 448, L.RBOS_F16_XPAIR) == 4 * 449 * 450 * 450
    assert lib.rbos_field_bytes(4, 4, 4, 6) == 0
    assert lib.rbos_code_scale(L.RBOS_F32_XPAIR, 0.0, 1.0, 0.0) == 1.0
    assert lib.rbos_code_scale(L.RBOS_BF16_XPAIR, -2.0 ** -16, 0.0, 0.0) == 2.0 ** 30
