"""Scene geometry for the synthetic BOS workloads.

Geometry follows the setup of Sec. 2.A (a room, a camera, and a back wall that is
either printed or lit by a projector) and the camera / projector arrangement of
Sec. 3.A (both looking along +y, projector offset +1 m in x from the camera). Units
are metres; the world frame has z up.

A `Scene` is plain data. Each consumer (GPU binding, oracle wrapper) marshals it into
its own C struct.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

Vec3 = Tuple[float, float, float]

ROOM_LO: Vec3 = (0.0, 0.0, 0.0)
ROOM_HI: Vec3 = (4.0, 4.0, 3.0)

WALL_PRINTED = 0
WALL_PROJECTOR = 1


@dataclasses.dataclass
class Scene:
    """One BOS acquisition: voxel grid + camera + back wall + integrator settings."""

    dims: Tuple[int, int, int]  # (nx, ny, nz) voxels
    box_lo: Vec3
    box_hi: Vec3
    cam_pos: Vec3
    cam_fwd: Vec3
    cam_right: Vec3
    cam_up: Vec3
    fov_x_deg: float
    width: int
    height: int
    wall_origin: Vec3
    wall_normal: Vec3
    wall_u: Vec3
    wall_v: Vec3
    wall_mode: int
    pat_w: int
    pat_h: int
    pat_extent_u: float = 0.0  # printed pattern: size on the wall (m)
    pat_extent_v: float = 0.0
    proj_pos: Vec3 = (0.0, 0.0, 0.0)
    proj_fwd: Vec3 = (0.0, 1.0, 0.0)
    proj_right: Vec3 = (1.0, 0.0, 0.0)
    proj_up: Vec3 = (0.0, 0.0, 1.0)
    proj_fov_x_deg: float = 60.0
    step: float = 0.0  # RK4 step h in the ray parameter t (metres)
    max_steps: int = 512
    ckpt_stride: int = 16
    tracer: int = 0  # 0: nonlinear (Eq. 1 coupled), 1: quasi-linear (forces on the entry line)
    spp: int = 1  # rays per pixel (Eq. 2 pixel integral; 1 = one ray through the pixel centre)
    seed: int = 0  # sub-pixel sample generator key
    radiometry: int = 0  # 1: weight each ray by |<n_w, v_w>| / |X_w - camera|
    name: str = ""

    @property
    def n_pixels(self) -> int:
        return self.width * self.height

    @property
    def voxel_size(self) -> Tuple[float, float, float]:
        return tuple((h - l) / n for l, h, n in zip(self.box_lo, self.box_hi, self.dims))

    def replace(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)


def _half_voxel_step(lo: Vec3, hi: Vec3, dims) -> float:
    return 0.5 * min((h - l) / n for l, h, n in zip(lo, hi, dims))


def scene_unit_box() -> Scene:
    """32^3 on a unit box; 64x64 pinhole camera 1.5 m in front; printed wall 0.5 m behind."""
    lo, hi, dims = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (32, 32, 32)
    wall_dist = 3.0  # camera (y=-1.5) to wall (y=1.5)
    extent = 2.0 * wall_dist * math.tan(math.radians(20.0))
    return Scene(
        dims=dims, box_lo=lo, box_hi=hi,
        cam_pos=(0.5, -1.5, 0.5), cam_fwd=(0.0, 1.0, 0.0), cam_right=(1.0, 0.0, 0.0),
        cam_up=(0.0, 0.0, 1.0), fov_x_deg=40.0, width=64, height=64,
        wall_origin=(0.5, 1.5, 0.5), wall_normal=(0.0, -1.0, 0.0),
        wall_u=(1.0, 0.0, 0.0), wall_v=(0.0, 0.0, 1.0),
        wall_mode=WALL_PRINTED, pat_w=256, pat_h=256,
        pat_extent_u=extent, pat_extent_v=extent,
        step=_half_voxel_step(lo, hi, dims), max_steps=128, ckpt_stride=16, name="unit_box",
    )


def scene_room(dims=(128, 128, 128), width=512, height=512, max_steps=512,
               ckpt_stride=16, pat=1024, name="room") -> Scene:
    """The 4 x 4 x 3 m room: camera at (2,-1.5,1.5) looking +y, projector +1 m in x,
    back wall on the room's far face y = 4 m."""
    lo, hi = ROOM_LO, ROOM_HI
    return Scene(
        dims=tuple(int(d) for d in dims), box_lo=lo, box_hi=hi,
        cam_pos=(2.0, -1.5, 1.5), cam_fwd=(0.0, 1.0, 0.0), cam_right=(1.0, 0.0, 0.0),
        cam_up=(0.0, 0.0, 1.0), fov_x_deg=40.0, width=int(width), height=int(height),
        wall_origin=(2.0, 4.0, 1.5), wall_normal=(0.0, -1.0, 0.0),
        wall_u=(1.0, 0.0, 0.0), wall_v=(0.0, 0.0, 1.0),
        wall_mode=WALL_PROJECTOR, pat_w=pat, pat_h=pat,
        proj_pos=(3.0, -1.5, 1.5), proj_fwd=(0.0, 1.0, 0.0), proj_right=(1.0, 0.0, 0.0),
        proj_up=(0.0, 0.0, 1.0), proj_fov_x_deg=60.0,
        step=_half_voxel_step(lo, hi, dims), max_steps=int(max_steps),
        ckpt_stride=int(ckpt_stride), name=name,
    )


def scene_room_512() -> Scene:
    return scene_room((128, 128, 128), 512, 512, 512, 16, name="room_512")


def scene_room_1024x768() -> Scene:
    return scene_room((128, 128, 128), 1024, 768, 512, 16, name="room_1024x768")


def scene_room_1m() -> Scene:
    """Headline workload: 128^3 room field, 1024 x 1024 = 1,048,576 rays."""
    return scene_room((128, 128, 128), 1024, 1024, 512, 16, name="room_1m")


def scene_room_256_3m() -> Scene:
    return scene_room((256, 256, 192), 2048, 1536, 1024, 16, name="room_256_3m")


def batch_max_steps(lo, hi, dims) -> int:
    diag = math.sqrt(sum((h - l) ** 2 for l, h in zip(lo, hi)))
    h = _half_voxel_step(lo, hi, dims)
    return 16 * int(math.ceil(1.1 * diag / h / 16.0))


def scenes_batch(n_scenes: int = 64, base_seed: int = 1000, dim_range=(48, 192),
              ray_range=(128, 1024)):
    """Batch of independent room scenes. Scene i draws, from seed base_seed + i and in
    this order: nx, ny, nz ~ U{dim_range}, then W, H ~ U{ray_range}, then its plume field
    (as `plumes_room`) from the same generator. Returns (scene, FieldSpec) pairs."""
    from .fields import plumes_room

    out = []
    for i in range(n_scenes):
        rng = np.random.default_rng(base_seed + i)
        dims = tuple(int(x) for x in rng.integers(dim_range[0], dim_range[1] + 1, size=3))
        w, h = (int(x) for x in rng.integers(ray_range[0], ray_range[1] + 1, size=2))
        sc = scene_room(dims, w, h, batch_max_steps(ROOM_LO, ROOM_HI, dims), 16, name=f"batch_{i}")
        out.append((sc, plumes_room(lo=ROOM_LO, hi=ROOM_HI, rng=rng)))
    return out


def scene_paper_geometry(dims=(64, 64, 64), sensor=100) -> Scene:
    """The acquisition geometry stated in Sec. 3.A-3.B: camera at (0.85,-29,1.5) m and
    projector at (1.85,-29,1.5) m, both looking +y with a long focal length; 100 x 100
    sensor; 64^3 reconstruction grid. The paper gives no field of view; 8 degrees makes
    the camera footprint at the far wall (33 m away) about 4.6 m wide, i.e. the room."""
    sc = scene_room(dims, sensor, sensor, 1024, 16, name="paper")
    return sc.replace(cam_pos=(0.85, -29.0, 1.5), proj_pos=(1.85, -29.0, 1.5),
                      fov_x_deg=8.0, proj_fov_x_deg=12.0)


def default_pixel_ids(scene: Scene) -> Optional[np.ndarray]:
    return None
