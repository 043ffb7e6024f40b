"""Seeded synthetic inputs for BOS ray tracing: scenes, temperature fields, wall patterns.

This module produces *input data only*: scene geometry (box, camera, wall, projector,
integrator settings), temperature fields T on voxel centres and wall / projector
patterns. It holds none of the method's arithmetic (no refractive-index map, no ray
tracing, no rendering); both the GPU path and the FP64 oracle consume what it makes.

The paper's own inputs (an OpenFOAM RANS field and a wavelet-noise projector
pattern, Sec. 3.A) are not available; seeded Gaussian hot plumes, a vertical
stratification and random patterns stand in for them.
"""

from .scenes import (  # noqa: F401
    Scene,
    scene_unit_box,
    scene_room,
    scene_room_512,
    scene_room_1024x768,
    scene_room_1m,
    scene_room_256_3m,
    scenes_batch,
    scene_paper_geometry,
    ROOM_LO,
    ROOM_HI,
)
from .fields import (  # noqa: F401
    Plume,
    plume_unit_box,
    plumes_room,
    temperature_grid,
    voxel_centres,
    T_AMBIENT,
)
from .patterns import binary_dots, blurred_noise  # noqa: F401
from .subsets import pixel_subset, strided_tiles  # noqa: F401
from .network import mlp_params, mlp_param_shapes, inlet_points, collocation_points  # noqa: F401
