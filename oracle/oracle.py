"""ctypes wrapper of the FP64 oracle (`bos_oracle.c`). Test infrastructure only.

The wrapper takes the plain-data `bos_inputs.Scene` and NumPy arrays and marshals
them into the oracle's own C structs; it shares nothing with the GPU binding.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bos_oracle.c")
_LIB = os.path.join(_HERE, "libbos_oracle.so")

RAY_MISSED_BOX, RAY_TRUNCATED, RAY_NO_WALL_HIT, RAY_NONFINITE, RAY_OFF_PATTERN = 1, 2, 4, 8, 16
CODE_F32, CODE_F16, CODE_BF16 = 0, 1, 2
FIELD_GRID, FIELD_HOMOGENEOUS, FIELD_LINEAR, FIELD_ETA2_LINEAR, FIELD_GAUSSIAN = 0, 1, 2, 3, 4
TRACER_NONLINEAR, TRACER_QUASILINEAR = 0, 1

D3 = C.c_double * 3


class _Field(C.Structure):
    _fields_ = [
        ("mode", C.c_int32), ("n", C.c_int32 * 3), ("lo", D3), ("hi", D3),
        ("delta", C.POINTER(C.c_double)), ("a", C.c_double), ("g", D3), ("c", D3),
        ("sigma", C.c_double), ("eps", C.c_double),
        ("pert_index", C.c_int64), ("pert_value", C.c_double),
    ]


class _Scene(C.Structure):
    _fields_ = [
        ("width", C.c_int32), ("height", C.c_int32),
        ("cam_pos", D3), ("cam_fwd", D3), ("cam_right", D3), ("cam_up", D3), ("fov_x_deg", C.c_double),
        ("wall_origin", D3), ("wall_normal", D3), ("wall_u", D3), ("wall_v", D3),
        ("wall_mode", C.c_int32), ("pat_w", C.c_int32), ("pat_h", C.c_int32),
        ("pat_extent_u", C.c_double), ("pat_extent_v", C.c_double),
        ("proj_pos", D3), ("proj_fwd", D3), ("proj_right", D3), ("proj_up", D3),
        ("proj_fov_x_deg", C.c_double),
        ("step", C.c_double), ("max_steps", C.c_int32), ("tracer", C.c_int32),
        ("spp", C.c_int32), ("seed", C.c_uint32), ("radiometry", C.c_int32),
        ("pattern", C.POINTER(C.c_double)),
    ]


def lib_path() -> str:
    return _LIB


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp -ffp-contract=off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.or_version.restype = C.c_int
        lib.or_threads.restype = C.c_int
        for name, args in {
            "or_delta_from_temperature": [P, C.c_int64, C.c_double, C.c_double, P],
            "or_delta_from_temperature_f32": [P, C.c_int64, C.c_float, C.c_float, P],
            "or_encode": [P, C.c_int64, C.c_int32, C.c_double, C.c_double, P],
            "or_decode": [P, C.c_int64, C.c_int32, C.c_double, C.c_double, P],
            "or_sample": [P, P, P, P, P],
            "or_camera_ray": [P, C.c_int32, P, P],
            "or_integrate": [P, P, P, C.c_double, C.c_int32, P, P],
            "or_integrate_quasi": [P, P, P, C.c_double, C.c_int32, P, P],
            "or_trace": [P, P, P, C.c_int32, P, P, P, P, P, P, P],
            "or_render": [P, P, C.c_int32, P, P, P, P],
            "or_render_pixels": [P, C.c_int32, P, P, P, P, P, P, P, P],
            "or_loss": [P, P, P, C.c_int32, P, P],
            "or_loss_pixels": [P, P, C.c_int32, C.c_int32, P, P, P, P, P, P, P],
            "or_adjoint": [P, P, P, C.c_int32, P, P, P, P],
            "or_tangent": [P, P, P, C.c_int32, P, P, P, P],
            "or_philox4x32": [P, P, P],
            "or_sample_offset": [C.c_uint32, C.c_int32, C.c_int32, P, P],
            "or_fd_voxels": [P, P, P, C.c_int32, P, P, C.c_int32, C.c_double, C.c_int32, P],
        }.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = C.c_int
        _lib = lib
    return _lib


def threads() -> int:
    return int(load().or_threads())


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc: int, name: str):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with code {rc}")


class Field:
    """An oracle field (keeps the backing array alive)."""

    def __init__(self, struct: _Field, keep=None):
        self.s = struct
        self._keep = keep

    @property
    def ref(self):
        return C.byref(self.s)

    def perturbed(self, index: int, value: float) -> "Field":
        s = _Field.from_buffer_copy(self.s)
        s.pert_index = index
        s.pert_value = value
        return Field(s, self._keep)


def grid_field(delta: np.ndarray, lo: Sequence[float], hi: Sequence[float]) -> Field:
    """Grid field from eta - 1 at voxel centres, array [nz][ny][nx]."""
    d = np.ascontiguousarray(delta, dtype=np.float64)
    nz, ny, nx = d.shape
    s = _Field()
    s.mode = FIELD_GRID
    s.n[:] = (nx, ny, nz)
    s.lo[:] = tuple(lo)
    s.hi[:] = tuple(hi)
    s.delta = d.ctypes.data_as(C.POINTER(C.c_double))
    s.pert_index = -1
    return Field(s, d)


def analytic_field(mode: int, lo, hi, a=0.0, g=(0.0, 0.0, 0.0), c=(0.0, 0.0, 0.0), sigma=1.0,
                   eps=0.0) -> Field:
    s = _Field()
    s.mode = mode
    s.n[:] = (0, 0, 0)
    s.lo[:] = tuple(lo)
    s.hi[:] = tuple(hi)
    s.a = a
    s.g[:] = tuple(g)
    s.c[:] = tuple(c)
    s.sigma = sigma
    s.eps = eps
    s.pert_index = -1
    return Field(s)


class _SceneHolder:
    def __init__(self, scene, pattern: Optional[np.ndarray]):
        s = _Scene()
        s.width, s.height = scene.width, scene.height
        for k in ("cam_pos", "cam_fwd", "cam_right", "cam_up", "wall_origin", "wall_normal",
                  "wall_u", "wall_v", "proj_pos", "proj_fwd", "proj_right", "proj_up"):
            getattr(s, k)[:] = tuple(float(x) for x in getattr(scene, k))
        s.fov_x_deg = scene.fov_x_deg
        s.proj_fov_x_deg = scene.proj_fov_x_deg
        s.wall_mode = scene.wall_mode
        s.pat_w, s.pat_h = scene.pat_w, scene.pat_h
        s.pat_extent_u, s.pat_extent_v = scene.pat_extent_u, scene.pat_extent_v
        s.step = scene.step
        s.max_steps = scene.max_steps
        s.tracer = getattr(scene, "tracer", TRACER_NONLINEAR)
        s.spp = getattr(scene, "spp", 1)
        s.seed = getattr(scene, "seed", 0)
        s.radiometry = getattr(scene, "radiometry", 0)
        self.pattern = None
        if pattern is not None:
            p = np.ascontiguousarray(pattern, dtype=np.float64)
            assert p.shape == (scene.pat_h, scene.pat_w), p.shape
            self.pattern = p
            s.pattern = p.ctypes.data_as(C.POINTER(C.c_double))
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)


def _ids(scene, pixel_ids):
    """(pixel id array or None, number of rays = samples per pixel x pixels)."""
    spp = getattr(scene, "spp", 1)
    if pixel_ids is None:
        return None, scene.width * scene.height * spp
    ids = np.ascontiguousarray(pixel_ids, dtype=np.int32)
    return ids, int(ids.size) * spp


# --- Sec. 2.A ---------------------------------------------------------------------------

def delta_from_temperature(T: np.ndarray, rho0G: float = 2.7e-4, T0: float = 293.0) -> np.ndarray:
    t = np.ascontiguousarray(T, dtype=np.float32)
    out = np.empty(t.shape, np.float64)
    _check(load().or_delta_from_temperature(_ptr(t), t.size, rho0G, T0, _ptr(out)), "delta")
    return out


def delta_from_temperature_f32(T: np.ndarray, rho0G: float = 2.7e-4, T0: float = 293.0) -> np.ndarray:
    t = np.ascontiguousarray(T, dtype=np.float32)
    out = np.empty(t.shape, np.float32)
    _check(load().or_delta_from_temperature_f32(_ptr(t), t.size, rho0G, T0, _ptr(out)), "delta_f32")
    return out


def encode(delta_f32: np.ndarray, code: int, scale: float = 1.0, offset: float = 0.0) -> np.ndarray:
    d = np.ascontiguousarray(delta_f32, dtype=np.float32)
    out = np.empty(d.shape, np.float32 if code == CODE_F32 else np.uint16)
    _check(load().or_encode(_ptr(d), d.size, code, scale, offset, _ptr(out)), "encode")
    return out


def decode(codes: np.ndarray, code: int, scale: float = 1.0, offset: float = 0.0) -> np.ndarray:
    q = np.ascontiguousarray(codes)
    out = np.empty(q.shape, np.float64)
    _check(load().or_decode(_ptr(q), q.size, code, scale, offset, _ptr(out)), "decode")
    return out


# --- sampler, camera, integrator ---------------------------------------------------------

def sample(field: Field, P):
    p = np.ascontiguousarray(P, dtype=np.float64)
    d = np.zeros(1)
    g = np.zeros(3)
    h = np.zeros(9)
    _check(load().or_sample(field.ref, _ptr(p), _ptr(d), _ptr(g), _ptr(h)), "sample")
    return float(d[0]), g, h.reshape(3, 3)


def camera_ray(scene, pixel: int):
    sh = _SceneHolder(scene, None)
    o = np.zeros(3)
    d = np.zeros(3)
    _check(load().or_camera_ray(sh.ref, pixel, _ptr(o), _ptr(d)), "camera_ray")
    return o, d


def integrate(field: Field, x0, v0, h: float, nsteps: int, quasi: bool = False):
    """nsteps steps from (x0, v0) with no box: nonlinear, or quasi-linear (forces on the
    line x0 + v0 t)."""
    x0 = np.ascontiguousarray(x0, np.float64)
    v0 = np.ascontiguousarray(v0, np.float64)
    x = np.zeros(3)
    v = np.zeros(3)
    fn = load().or_integrate_quasi if quasi else load().or_integrate
    _check(fn(field.ref, _ptr(x0), _ptr(v0), h, nsteps, _ptr(x), _ptr(v)), "integrate")
    return x, v


# --- forward, render, loss -----------------------------------------------------------------

def trace(field: Field, scene, pixel_ids=None, want_exit=False):
    """Returns dict(uv, duv, n_steps, status, vdir, path[, exit_xv]) per ray (ray r = sample
    r // P of pixel r % P; vdir the unit direction at the wall, path the length of the
    ray path from the camera centre to the wall hit)."""
    ids, n = _ids(scene, pixel_ids)
    sh = _SceneHolder(scene, None)
    uv = np.empty((n, 2))
    duv = np.empty((n, 2))
    ns = np.empty(n, np.int32)
    st = np.empty(n, np.uint8)
    vd = np.empty((n, 3))
    pl = np.empty(n)
    ex = np.empty((n, 6)) if want_exit else None
    _check(load().or_trace(field.ref, sh.ref, _ptr(ids), n, _ptr(uv), _ptr(duv), _ptr(ns), _ptr(st),
                           _ptr(ex), _ptr(vd), _ptr(pl)), "trace")
    out = dict(uv=uv, duv=duv, n_steps=ns, status=st, vdir=vd, path=pl)
    if want_exit:
        out["exit_xv"] = ex
    return out


def render(scene, pattern: np.ndarray, uv: np.ndarray, status: np.ndarray):
    """Wall luminance per ray and dI/d(u, v); returns (image, dI_duv, status)."""
    sh = _SceneHolder(scene, pattern)
    uv = np.ascontiguousarray(uv, np.float64)
    st = np.array(status, dtype=np.uint8, copy=True)
    n = uv.shape[0]
    img = np.empty(n)
    dI = np.empty((n, 2))
    _check(load().or_render(sh.ref, None, n, _ptr(uv), _ptr(st), _ptr(img), _ptr(dI)), "render")
    return img, dI, st


def render_pixels(scene, pattern: np.ndarray, uv: np.ndarray, status: np.ndarray, vdir=None, path=None):
    """Eq. (2) per pixel: dict(image [P], dI_duv [n_rays, 2], dI_ddir [n_rays, 3],
    dI_dpath [n_rays], status)."""
    sh = _SceneHolder(scene, pattern)
    uv = np.ascontiguousarray(uv, np.float64)
    st = np.array(status, dtype=np.uint8, copy=True)
    n = uv.shape[0]
    spp = getattr(scene, "spp", 1)
    P = n // spp
    vd = None if vdir is None else np.ascontiguousarray(vdir, np.float64)
    pl = None if path is None else np.ascontiguousarray(path, np.float64)
    img = np.empty(P)
    dI = np.empty((n, 2))
    dId = np.empty((n, 3))
    dIp = np.empty(n)
    _check(load().or_render_pixels(sh.ref, P, _ptr(uv), _ptr(vd), _ptr(pl), _ptr(st), _ptr(img), _ptr(dI),
                                   _ptr(dId), _ptr(dIp)), "render_pixels")
    return dict(image=img, dI_duv=dI, dI_ddir=dId, dI_dpath=dIp, status=st)


def loss_pixels(image, target, spp, dI_duv, dI_ddir=None, dI_dpath=None):
    """L_BOS over pixels, and per ray dL/d(u, v), dL/d(vdir) and dL/d(path) (the last two
    None when their inputs are)."""
    image = np.ascontiguousarray(image, np.float64)
    target = np.ascontiguousarray(target, np.float64)
    dI_duv = np.ascontiguousarray(dI_duv, np.float64)
    dId = None if dI_ddir is None else np.ascontiguousarray(dI_ddir, np.float64)
    dIp = None if dI_dpath is None else np.ascontiguousarray(dI_dpath, np.float64)
    P = image.size
    L = np.zeros(1)
    g = np.empty((P * spp, 2))
    gd = np.empty((P * spp, 3)) if dId is not None else None
    gp = np.empty(P * spp) if dIp is not None else None
    _check(load().or_loss_pixels(_ptr(image), _ptr(target), P, spp, _ptr(dI_duv), _ptr(dId), _ptr(dIp), _ptr(L),
                                 _ptr(g), _ptr(gd), _ptr(gp)), "loss_pixels")
    return float(L[0]), g, gd, gp


def philox4x32(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.empty(4, np.uint32)
    _check(load().or_philox4x32(_ptr(c), _ptr(k), _ptr(out)), "philox")
    return out


def sample_offset(seed: int, pixel: int, sample: int):
    ox, oy = C.c_double(), C.c_double()
    _check(load().or_sample_offset(seed, pixel, sample, C.byref(ox), C.byref(oy)), "sample_offset")
    return ox.value, oy.value


def loss(image, target, dI_duv):
    image = np.ascontiguousarray(image, np.float64)
    target = np.ascontiguousarray(target, np.float64)
    dI_duv = np.ascontiguousarray(dI_duv, np.float64)
    n = image.size
    L = np.zeros(1)
    g = np.empty((n, 2))
    _check(load().or_loss(_ptr(image), _ptr(target), _ptr(dI_duv), n, _ptr(L), _ptr(g)), "loss")
    return float(L[0]), g


# --- derivatives ---------------------------------------------------------------------------

def adjoint(field: Field, scene, dL_duv, pixel_ids=None, dL_ddir=None, dL_dpath=None):
    ids, n = _ids(scene, pixel_ids)
    sh = _SceneHolder(scene, None)
    lam = np.ascontiguousarray(dL_duv, np.float64).reshape(n, 2)
    lam_d = None if dL_ddir is None else np.ascontiguousarray(dL_ddir, np.float64).reshape(n, 3)
    lam_p = None if dL_dpath is None else np.ascontiguousarray(dL_dpath, np.float64).reshape(n)
    nx, ny, nz = field.s.n
    g = np.zeros((nz, ny, nx))
    _check(load().or_adjoint(field.ref, sh.ref, _ptr(ids), n, _ptr(lam), _ptr(lam_d), _ptr(lam_p), _ptr(g)),
           "adjoint")
    return g


def tangent(field: Field, scene, vfield, pixel_ids=None, with_dir=False):
    """d(u, v) per ray; with_dir: (d(u, v), d vdir, d path)."""
    ids, n = _ids(scene, pixel_ids)
    sh = _SceneHolder(scene, None)
    vf = np.ascontiguousarray(vfield, np.float64)
    out = np.empty((n, 2))
    od = np.empty((n, 3)) if with_dir else None
    op = np.empty(n) if with_dir else None
    _check(load().or_tangent(field.ref, sh.ref, _ptr(ids), n, _ptr(vf), _ptr(out), _ptr(od), _ptr(op)), "tangent")
    return (out, od, op) if with_dir else out


def fd_voxels(field: Field, scene, pattern, target, voxels, h=1e-7, locked=True, pixel_ids=None):
    ids, n = _ids(scene, pixel_ids)
    sh = _SceneHolder(scene, pattern)
    tg = np.ascontiguousarray(target, np.float64).reshape(n // getattr(scene, "spp", 1))
    vx = np.ascontiguousarray(voxels, np.int64)
    out = np.empty(vx.size)
    _check(load().or_fd_voxels(field.ref, sh.ref, _ptr(ids), n, _ptr(tg), _ptr(vx), vx.size, h,
                               1 if locked else 0, _ptr(out)), "fd_voxels")
    return out
