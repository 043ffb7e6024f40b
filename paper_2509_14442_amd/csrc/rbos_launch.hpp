// rbos_launch.hpp -- host-side launch descriptors passed from the C ABI to the kernel
// translation units.
#pragma once

#include <hip/hip_runtime.h>

namespace rbos {

struct SceneDev;

struct LaunchPlan {
  const SceneDev* scenes;   // device scene table
  int n_scenes;
  int total_tiles;          // sum of per-scene 64-ray tiles
  int wpb;                  // wavefronts per block
  int dtype;                // storage type shared by all scenes of the call
  int persistent;           // 1: persistent blocks + per-XCD tile queues
  int blocks_per_cu;        // persistent: resident blocks per compute unit; 0 = the kernel's occupancy limit
  int n_cus;                // compute units of the device
  unsigned int* queues;     // 8 counters (zeroed before the launch)
  int ckpt_k;               // checkpoint stride shared by all scenes (adjoint)
  int tracer;               // shared by all scenes: 0 nonlinear, 1 quasi-linear
  int total_render_blocks;  // render: sum of per-scene blocks
  float* partials;          // render: per-block partial loss sums
  int* tile_cost;           // adjoint, persistent: longest ray of each tile (steps)
  int* tile_order;          // adjoint, persistent: processing order of the tiles
  int order_shift;          // cost >> order_shift is the sort key (< 1024)
};

// Grid of a persistent kernel: blocks_per_cu blocks on every compute unit, or as many as
// the kernel's registers and LDS let reside at once.
template <class Kernel>
inline int persistent_grid(Kernel kernel, const LaunchPlan& P, size_t lds_bytes) {
  int bpc = P.blocks_per_cu;
  if (bpc <= 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(kernel), 64 * P.wpb,
                                                     lds_bytes) != hipSuccess || n < 1)
      n = 1;
    bpc = n;
  }
  return bpc * P.n_cus;
}

hipError_t launch_trace_fwd(const LaunchPlan& P, hipStream_t stream);
hipError_t launch_render(const LaunchPlan& P, hipStream_t stream);
hipError_t launch_trace_adj(const LaunchPlan& P, hipStream_t stream);
// persistent adjoint: fill P.tile_order from the forward's step counts
hipError_t launch_tile_order(const LaunchPlan& P, hipStream_t stream);
hipError_t launch_field_pack(int nx, int ny, int nz, const float* src, int from_temperature, float rho0G, float T0,
                             int dtype, float scale, float offset, void* field, hipStream_t stream);
hipError_t launch_fill_u32(unsigned int* p, unsigned int value, int n, hipStream_t stream);
hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t stream);

}  // namespace rbos
