// trace_fwd.hip -- forward ray tracing (Sec. 2.B, Eq. 1): one ray per lane, 64-ray
// tiles per wavefront, every scene of a batch in one launch.
#include "rbos_device.hpp"
#include "rbos_launch.hpp"

namespace rbos {

// Trace one ray; writes its outputs. With checkpoints the buffer holds, component-major
// (component c of the ray at [c * ckpt_pad + ckpt_entry]): the ray header (see
// store_ray_header), then the states (d, e) before steps k, 2k, ... (6 components per
// slot).
template <int DT, bool QL>
__device__ __forceinline__ void trace_one(const SceneDev& S, int r, int pix, int smp) {
  int n = 0;
  unsigned char status = 0;
  float uvd[2] = {0.0f, 0.0f};
  bool ok = true;
  bool entered;
  RayBase B;
  Cell C;
  float e_end[3] = {0.0f, 0.0f, 0.0f};  // velocity deviation of the last state
  {
    Ray R;
    camera_ray(S, pix, smp, R.dir);
    df t_in;
    entered = box_entry(S, R.dir, t_in);
    if (entered) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        df x = dd_add(S.cam_pos[a], dd_mul(t_in, R.dir[a]));
        R.U0[a] = dd_add_f(dd_mul(dd_sub(x, S.lo[a]), S.inv_vox[a]), 0.5f);
      }
      make_base<DT>(S, R, B, C);
    }
  }
  if (!entered) {
    status |= RAY_MISSED_BOX;
  } else {
    State st;
    state_at_step(B, 0, st);
#pragma unroll
    for (int a = 0; a < 3; ++a) { st.d[a] = 0.0f; st.e[a] = 0.0f; }
    // checkpoint slot s holds the state after (s + 1) K steps
    const int q = ckpt_entry(S, r, pix, smp);
    float* ck = S.ckpt ? S.ckpt + (size_t)RAY_HEADER * S.ckpt_pad + (size_t)q : nullptr;
    const size_t slot_stride = 6 * (size_t)S.ckpt_pad;
    bool exited = false;
    // after each step: count it, stop on a non-finite state or outside the box. After a
    // Sharma step a non-finite position locates as NaN (outside), so only the velocity is
    // tested every step and the whole state once the ray stops.
    auto stop = [&]() {
      ++n;
      if (!isfinite((st.e[0] + st.e[1]) + st.e[2]) || outside_located(S, st, C)) {
        exited = true;
        if (!state_finite(st)) status |= RAY_NONFINITE;
      }
      return exited;
    };
    if constexpr (QL) {
      float Kc[3];  // force at the current point of the entry line
      force_at<DT>(S, C, Kc);
      while (n < S.max_steps) {
        ql_step<DT>(S, B, st, Kc);
        ++n;
        if (!state_finite(st)) {
          status |= RAY_NONFINITE;
          exited = true;
        } else if (outside_box(S, B, st)) {
          exited = true;
        }
        if (exited) break;
      }
    } else if (!ck) {
      while (n < S.max_steps) {
        sharma_step<DT>(S, B, st, C);
        if (stop()) break;
      }
    } else {
      // Segments of K steps; every segment after the first starts with a step whose start
      // state is stored. That step is a copy of its own with unconditional stores, issued
      // after its first gather (see NoIssue): in one loop with a branch around the stores,
      // the wait for the next gather at the branch's join would have to cover them.
      const int K = S.ckpt_k;
      int until = min(K, S.max_steps);
      while (!exited) {
        while (n < until) {
          sharma_step<DT>(S, B, st, C);
          if (stop()) break;
        }
        if (exited || n >= S.max_steps) break;
        sharma_step<DT>(S, B, st, C, NoRecord(), [&]() {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            gst_stream(ck + (size_t)a * S.ckpt_pad, st.d[a]);
            gst_stream(ck + (size_t)(3 + a) * S.ckpt_pad, st.e[a]);
          }
        });
        ck += slot_stride;
        if (stop()) break;
        until = min(n - 1 + K, S.max_steps);
      }
    }
    if (!exited) status |= RAY_TRUNCATED;
#pragma unroll
    for (int a = 0; a < 3; ++a) e_end[a] = st.e[a];
    if (!(status & RAY_NONFINITE)) {
      float dX[3], s = 0.0f;
      const bool hit = wall_deflection(S, B, st, dX, &s);
      if (S.ckpt) store_ray_header(S, ckpt_entry(S, r, pix, smp), B, st, s);
      if (hit) {
        uvd[0] = dX[0] * S.wall_u_f[0] + dX[1] * S.wall_u_f[1] + dX[2] * S.wall_u_f[2];
        uvd[1] = dX[0] * S.wall_v_f[0] + dX[1] * S.wall_v_f[1] + dX[2] * S.wall_v_f[2];
      } else {
        status |= RAY_NO_WALL_HIT;
        ok = false;
      }
    } else {
      ok = false;
    }
  }
  // the undeflected camera ray's wall hit, recomputed here rather than kept live
  df dir[3], uv0[2];
  camera_ray(S, pix, smp, dir);
  const bool wall0 = wall_hit_straight(S, dir, uv0);
  if (!wall0 && !(status & RAY_NONFINITE)) {
    // the camera ray itself never reaches the wall: treat the hit as missing
    status |= RAY_NO_WALL_HIT;
    ok = false;
  }
  float u, v;
  if (ok) {
    u = dd_to_f(dd_add_f(uv0[0], uvd[0]));
    v = dd_to_f(dd_add_f(uv0[1], uvd[1]));
  } else {
    u = v = __builtin_nanf("");
    uvd[0] = uvd[1] = __builtin_nanf("");
  }
  gst(S.uv + 2 * (size_t)r, u);
  gst(S.uv + 2 * (size_t)r + 1, v);
  if (S.duv) {
    gst(S.duv + 2 * (size_t)r, uvd[0]);
    gst(S.duv + 2 * (size_t)r + 1, uvd[1]);
  }
  gst(S.n_steps + r, n);
  gst(S.status + r, status);
  if (S.wall_dir) {
    // unit direction at the wall: the exit velocity V + e (world units), or the camera
    // ray's for rays that never enter the box
    float w[3];
    if (status & RAY_NONFINITE) {
      w[0] = w[1] = w[2] = __builtin_nanf("");
    } else if (entered) {
      float n2 = 0.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        w[a] = fmaf(e_end[a], S.vox[a], B.V[a]);
        n2 = fmaf(w[a], w[a], n2);
      }
      const float inv = 1.0f / sqrtf(n2);
#pragma unroll
      for (int a = 0; a < 3; ++a) w[a] *= inv;
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) w[a] = dd_to_f(dir[a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) gst(S.wall_dir + 3 * (size_t)r + a, w[a]);
  }
}

// Held to 64 registers for 8 wavefronts per SIMD (68 would allow 7): the trace without
// checkpoints runs 3 % faster; with checkpoints it is unchanged.
template <int DT, bool QL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_trace_fwd(
    const SceneDev* __restrict__ scenes, int n_scenes, int total_tiles, int wpb, int nblocks) {
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int gtile = xcd_remap(blockIdx.x, nblocks) * wpb + wave;
  if (gtile >= total_tiles) return;
  const int si = find_scene(scenes, n_scenes, gtile);
  const SceneDev& S = scenes[si];
  const int tile = gtile - S.tile_begin;
  int r, pix, smp;
  if (!tile_ray(S, tile, lane, r, pix, smp)) return;
  trace_one<DT, QL>(S, r, pix, smp);
}

// Persistent form: blocks pull tiles from per-XCD queues (every 8th run of tiles), and
// steal from the other XCDs' queues once their own is drained.
template <int DT, bool QL>
__global__ __launch_bounds__(256) void k_trace_fwd_persistent(const SceneDev* __restrict__ scenes, int n_scenes,
                                                              int total_tiles, unsigned int* __restrict__ queues) {
  const int lane = threadIdx.x & 63;
  const int xcd = blockIdx.x & 7;
  for (int q = 0; q < 8; ++q) {
    const int qx = (xcd + q) & 7;
    int q_begin, q_end;
    xcd_tile_range(total_tiles, qx, q_begin, q_end);
    while (true) {
      int t = 0;
      if (lane == 0) t = (int)atomicAdd(&queues[qx], 1u);
      t = wave_uniform(t);  // lane 0's claim (all lanes active)
      if (t >= q_end - q_begin) break;
      t = xcd_tile(total_tiles, qx, t);
      const int si = find_scene(scenes, n_scenes, t);
      const SceneDev& S = scenes[si];
      const int tile = t - S.tile_begin;
      int r, pix, smp;
      if (tile_ray(S, tile, lane, r, pix, smp)) trace_one<DT, QL>(S, r, pix, smp);
    }
  }
}

template <int DT, bool QL>
static hipError_t launch_fwd_t(const LaunchPlan& P, hipStream_t stream) {
  const dim3 block(64 * P.wpb);
  if (P.persistent) {
    const dim3 grid(persistent_grid(k_trace_fwd_persistent<DT, QL>, P, 0));
    hipLaunchKernelGGL((k_trace_fwd_persistent<DT, QL>), grid, block, 0, stream, P.scenes, P.n_scenes,
                       P.total_tiles, P.queues);
  } else {
    const int nblocks = (P.total_tiles + P.wpb - 1) / P.wpb;
    hipLaunchKernelGGL((k_trace_fwd<DT, QL>), dim3(nblocks), block, 0, stream, P.scenes, P.n_scenes, P.total_tiles,
                       P.wpb, nblocks);
  }
  return hipGetLastError();
}

template <int DT>
static hipError_t launch_fwd_dt(const LaunchPlan& P, hipStream_t stream) {
  return P.tracer == 1 ? launch_fwd_t<DT, true>(P, stream) : launch_fwd_t<DT, false>(P, stream);
}

hipError_t launch_trace_fwd(const LaunchPlan& P, hipStream_t stream) {
  if (P.total_tiles == 0) return hipSuccess;
  switch (P.dtype) {
    case DT_F32: return launch_fwd_dt<DT_F32>(P, stream);
    case DT_F16: return launch_fwd_dt<DT_F16>(P, stream);
    case DT_BF16: return launch_fwd_dt<DT_BF16>(P, stream);
    case DT_F32_XPAIR: return launch_fwd_dt<DT_F32_XPAIR>(P, stream);
    case DT_F16_XPAIR: return launch_fwd_dt<DT_F16_XPAIR>(P, stream);
    default: return launch_fwd_dt<DT_BF16_XPAIR>(P, stream);
  }
}

}  // namespace rbos
