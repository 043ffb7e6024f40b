"""MI355X-native BOS ray tracing: forward, rendering, loss and adjoint of single-view
background-oriented-schlieren tomography (Eq. 1 with Sharma RK4 on a voxel grid), as
hand-written gfx950 HIP kernels behind the C ABI in include/rbos.h.

The C library (librbos.so) is built in-tree by `paper_2509_14442_amd.build`; importing
this package does not load it. `api` holds the torch binding.
"""

__all__ = ["api", "build"]
