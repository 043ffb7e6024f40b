"""FP64 CPU oracle for single-view BOS ray tracing.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library. See `bos_oracle.c` for what
it computes and the paper sections it follows.
"""

from .oracle import (  # noqa: F401
    build,
    lib_path,
    load,
    Field,
    grid_field,
    analytic_field,
    delta_from_temperature,
    delta_from_temperature_f32,
    encode,
    decode,
    sample,
    camera_ray,
    integrate,
    trace,
    render,
    render_pixels,
    loss,
    loss_pixels,
    philox4x32,
    sample_offset,
    adjoint,
    tangent,
    fd_voxels,
    threads,
    RAY_MISSED_BOX,
    RAY_TRUNCATED,
    RAY_NO_WALL_HIT,
    RAY_NONFINITE,
    RAY_OFF_PATTERN,
    CODE_F32,
    CODE_F16,
    CODE_BF16,
)
