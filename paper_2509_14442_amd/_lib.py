"""ctypes declarations of the librbos C ABI (include/rbos.h). Argument marshalling only."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbos.so")

D3 = C.c_double * 3

RBOS_F32, RBOS_F16, RBOS_BF16 = 0, 1, 2
RBOS_F32_XPAIR, RBOS_F16_XPAIR, RBOS_BF16_XPAIR = 3, 4, 5
RBOS_WALL_PRINTED, RBOS_WALL_PROJECTOR = 0, 1
RBOS_TRACER_NONLINEAR, RBOS_TRACER_QUASILINEAR = 0, 1
NOALLOC_SCRATCH_BYTES = 4 << 20  # RBOS_NOALLOC_SCRATCH_BYTES
RAY_MISSED_BOX, RAY_TRUNCATED, RAY_NO_WALL_HIT, RAY_NONFINITE, RAY_OFF_PATTERN = 1, 2, 4, 8, 16

STATUS = {
    0: "RBOS_OK", -1: "RBOS_E_NULL", -2: "RBOS_E_SHAPE", -3: "RBOS_E_RANGE", -4: "RBOS_E_DTYPE",
    -5: "RBOS_E_WORKSPACE", -6: "RBOS_E_HIP", -7: "RBOS_E_UNSUPPORTED",
}


class rbos_scene(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("box_lo", D3), ("box_hi", D3),
        ("dtype", C.c_int32), ("enc_scale", C.c_double), ("enc_offset", C.c_double),
        ("field", C.c_void_p),
        ("cam_pos", D3), ("cam_fwd", D3), ("cam_right", D3), ("cam_up", D3),
        ("cam_fov_x_deg", C.c_double),
        ("width", C.c_int32), ("height", C.c_int32),
        ("pixel_ids", C.c_void_p), ("n_pixels", C.c_int32),
        ("wall_origin", D3), ("wall_normal", D3), ("wall_u", D3), ("wall_v", D3),
        ("wall_mode", C.c_int32),
        ("pattern", C.c_void_p), ("pat_w", C.c_int32), ("pat_h", C.c_int32),
        ("pat_extent_u", C.c_double), ("pat_extent_v", C.c_double),
        ("proj_pos", D3), ("proj_fwd", D3), ("proj_right", D3), ("proj_up", D3),
        ("proj_fov_x_deg", C.c_double),
        ("step", C.c_double), ("max_steps", C.c_int32), ("ckpt_stride", C.c_int32), ("tracer", C.c_int32),
        ("spp", C.c_int32), ("seed", C.c_uint32), ("radiometry", C.c_int32),
    ]


class rbos_trace_out(C.Structure):
    _fields_ = [("wall_uv", C.c_void_p), ("wall_duv", C.c_void_p), ("n_steps", C.c_void_p),
                ("status", C.c_void_p), ("ckpt", C.c_void_p), ("wall_dir", C.c_void_p)]


class rbos_render_io(C.Structure):
    _fields_ = [("target", C.c_void_p), ("image", C.c_void_p), ("dL_duv", C.c_void_p), ("loss", C.c_void_p),
                ("dL_ddir", C.c_void_p)]


class rbos_adjoint_io(C.Structure):
    _fields_ = [("dL_duv", C.c_void_p), ("grad", C.c_void_p), ("dL_ddir", C.c_void_p)]


class rbos_launch(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("waves_per_block", C.c_int32),
                ("persistent", C.c_int32), ("blocks_per_cu", C.c_int32)]


class rbos_mlp(C.Structure):
    _fields_ = [("width", C.c_int32), ("depth", C.c_int32), ("params", C.c_void_p), ("box_lo", D3),
                ("box_hi", D3)]


class rbos_pde(C.Structure):
    _fields_ = [("Re", C.c_double), ("Pe", C.c_double), ("Ri", C.c_double), ("L", C.c_double), ("gamma", D3)]


STRUCTS = [rbos_scene, rbos_trace_out, rbos_render_io, rbos_adjoint_io, rbos_launch, rbos_mlp, rbos_pde]

EXPORTS = [
    "rbos_version", "rbos_last_error", "rbos_field_bytes", "rbos_field_from_temperature",
    "rbos_field_encode", "rbos_code_scale", "rbos_code_scale_temperature", "rbos_ckpt_bytes", "rbos_workspace_bytes", "rbos_trace_forward",
    "rbos_render", "rbos_trace_adjoint", "rbos_trace_adjoint_noalloc", "rbos_struct_layout",
    "rbos_mlp_param_count", "rbos_mlp_workspace_bytes", "rbos_mlp_forward", "rbos_mlp_backward", "rbos_mlp_bos_seed",
    "rbos_mlp_fit_workspace_bytes", "rbos_mlp_fit_seed", "rbos_mlp_pde_workspace_bytes", "rbos_mlp_pde_loss",
]

_lib = None


class RbosError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load librbos.so (built in-tree by `paper_2509_14442_amd.build`); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2509_14442_amd.build` "
                           "(there is no fallback implementation)")
    lib = C.CDLL(path)
    P, I32, SZ = C.c_void_p, C.c_int32, C.c_size_t
    sig = {
        "rbos_version": ([], C.c_int),
        "rbos_last_error": ([], C.c_char_p),
        "rbos_field_bytes": ([I32, I32, I32, I32], SZ),
        "rbos_field_from_temperature": ([I32, I32, I32, P, C.c_double, C.c_double, I32, C.c_double,
                                         C.c_double, P, P], C.c_int),
        "rbos_field_encode": ([I32, I32, I32, P, I32, C.c_double, C.c_double, P, P], C.c_int),
        "rbos_code_scale": ([I32, C.c_double, C.c_double, C.c_double], C.c_double),
        "rbos_code_scale_temperature": ([I32, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double],
                                        C.c_double),
        "rbos_ckpt_bytes": ([C.POINTER(rbos_scene)], SZ),
        "rbos_workspace_bytes": ([C.POINTER(rbos_scene), I32], SZ),
        "rbos_trace_forward": ([C.POINTER(rbos_scene), I32, C.POINTER(rbos_trace_out),
                                C.POINTER(rbos_launch), P, SZ, P], C.c_int),
        "rbos_render": ([C.POINTER(rbos_scene), I32, C.POINTER(rbos_trace_out), C.POINTER(rbos_render_io),
                         P, SZ, P], C.c_int),
        "rbos_trace_adjoint": ([C.POINTER(rbos_scene), I32, C.POINTER(rbos_trace_out),
                                C.POINTER(rbos_adjoint_io), C.POINTER(rbos_launch), P, SZ, P], C.c_int),
        "rbos_trace_adjoint_noalloc": ([C.POINTER(rbos_scene), I32, C.POINTER(rbos_trace_out),
                                        C.POINTER(rbos_adjoint_io), C.POINTER(rbos_launch), P], C.c_int),
        "rbos_struct_layout": ([I32, C.POINTER(C.c_size_t), I32], SZ),
        "rbos_mlp_param_count": ([I32, I32], SZ),
        "rbos_mlp_workspace_bytes": ([I32, I32, C.c_int64], SZ),
        "rbos_mlp_forward": ([C.POINTER(rbos_mlp), P, C.c_int64, P, P, P, C.c_double, C.c_double, P, SZ, P],
                             C.c_int),
        "rbos_mlp_backward": ([C.POINTER(rbos_mlp), P, C.c_int64, P, P, P, P, SZ, P], C.c_int),
        "rbos_mlp_bos_seed": ([C.c_int64, P, P, C.c_double, C.c_double, C.c_double, P, P], C.c_int),
        "rbos_mlp_fit_workspace_bytes": ([C.c_int64], SZ),
        "rbos_mlp_fit_seed": ([C.c_int64, P, P, C.POINTER(C.c_double), P, P, P, SZ, P], C.c_int),
        "rbos_mlp_pde_workspace_bytes": ([I32, I32, C.c_int64], SZ),
        "rbos_mlp_pde_loss": ([C.POINTER(rbos_mlp), C.POINTER(rbos_pde), P, C.c_int64, P, P, P, P, SZ, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(rc: int):
    if rc != 0:
        msg = load().rbos_last_error()
        raise RbosError(rc, msg.decode() if msg else "")
    return rc
