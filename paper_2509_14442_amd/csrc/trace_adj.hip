// trace_adj.hip -- Sec. 2.D: exact gradient of L_BOS with respect to eta - 1 per voxel,
// back-propagated through the wall step and every Sharma step of Eq. (1).
//
// Per wavefront (64 rays of one tile), segments between checkpoints are processed from
// the last to the first, aligned on the step index so that the tile's rays move through
// the same cells together. A segment is replayed forward from its checkpoint in chunks
// of KS steps whose states stay in registers, then reversed step by step. Each sample's
// eight corner contributions are merged per lane while the ray stays in one cell; on a
// cell change the lanes leaving the same cell are summed across the wavefront and one
// FP64 atomic per corner goes to the gradient.
#include "rbos_device.hpp"
#include "rbos_launch.hpp"

namespace rbos {

// Everything the reverse sweep needs about one sample.
struct SampleRev {
  Cell C;
  float g[3], H[3];  // code-unit gradient and mixed second derivatives (unmasked)
  float eta;         // 1 + delta
};

template <int DT>
__device__ __forceinline__ void sample_rev(const SceneDev& S, const Cell& C, SampleRev& R, float K[3]) {
  float c[8];
  fetch_cell<DT>(S.field, cell_index(S, C), c);
  float q;
  trilinear_h(c, C.f, q, R.g, R.H);
  R.eta = fmaf(q, S.dec, S.one_plus_off);
  R.C = C;
#pragma unroll
  for (int a = 0; a < 3; ++a) K[a] = R.eta * (R.g[a] * (C.m[a] * S.km[a]));
}

// Reverse of K = force(P) for an adjoint v = dL/dK: returns p = dL/dP (grid units) and
// the 8 corner contributions dL/d(delta_c):
//   w_a = v_a m_a km_a,  sigma = sum_a w_a g_a,
//   p_b = m_b (dec g_b sigma + eta sum_{a != b} w_a H_ab),
//   dL/d delta_c = w_c sigma + (eta / dec) sum_a w_a dw_c/du_a.
__device__ __forceinline__ void force_rev(const SceneDev& S, const SampleRev& R, const float v[3], float p[3],
                                          float contrib[8]) {
  const float* m = R.C.m;
  float w0 = v[0] * (m[0] * S.km[0]), w1 = v[1] * (m[1] * S.km[1]), w2 = v[2] * (m[2] * S.km[2]);
  float sigma = fmaf(w0, R.g[0], fmaf(w1, R.g[1], w2 * R.g[2]));
  float ds = S.dec * sigma;
  // H = (H_xy, H_xz, H_yz)
  p[0] = m[0] * fmaf(ds, R.g[0], R.eta * fmaf(w1, R.H[0], w2 * R.H[1]));
  p[1] = m[1] * fmaf(ds, R.g[1], R.eta * fmaf(w0, R.H[0], w2 * R.H[2]));
  p[2] = m[2] * fmaf(ds, R.g[2], R.eta * fmaf(w0, R.H[1], w1 * R.H[2]));
  // corner weights: w = X_i Y_j Z_k with X_0 = 1 - fx, X_1 = fx; dX_i/du = -1, +1
  const float fx = R.C.f[0], fy = R.C.f[1], fz = R.C.f[2];
  const float X[2] = {1.0f - fx, fx}, Y[2] = {1.0f - fy, fy}, Z[2] = {1.0f - fz, fz};
  const float ed = R.eta / S.dec;
  const float Wx = w0 * ed, Wy = w1 * ed, Wz = w2 * ed;
  const float alpha[2] = {fmaf(X[0], sigma, -Wx), fmaf(X[1], sigma, Wx)};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      float yz = Y[j] * Z[k];
      float sy = j ? Wy : -Wy, sz = k ? Wz : -Wz;
      float beta = fmaf(sy, Z[k], sz * Y[j]);
#pragma unroll
      for (int i = 0; i < 2; ++i) contrib[i + 2 * j + 4 * k] = fmaf(yz, alpha[i], X[i] * beta);
    }
  }
}

// Per-lane merge of corner contributions by cell, flushed across the wavefront.
struct Accum {
  float acc[8];
  int cell;  // voxel index of the cell's lower corner, -1 when empty
};

__device__ __forceinline__ int voxel_of(const SceneDev& S, const Cell& C) {
  return C.i[0] + S.n[0] * (C.i[1] + S.n[1] * C.i[2]);
}

// Add the accumulators of lanes with `sel` to the gradient: lanes that hold the same
// cell are summed across the wavefront; lanes 0-7 then add one corner each (FP64).
// Must be called with all 64 lanes active.
__device__ __forceinline__ void flush(const SceneDev& S, Accum& A, bool sel, int lane) {
  unsigned long long pend = __ballot(sel);
  const int nx = S.n[0], nxy = S.n[0] * S.n[1];
  while (pend) {
    const int leader = __ffsll((long long)pend) - 1;
    const int c = __builtin_amdgcn_readlane(A.cell, leader);
    const bool mine = sel && A.cell == c;
    float s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = wave_sum(mine ? A.acc[k] : 0.0f);
    if (lane < 8) {
      float val = s[0];
#pragma unroll
      for (int k = 1; k < 8; ++k) val = (lane == k) ? s[k] : val;
      const int off = (lane & 1) + ((lane >> 1) & 1) * nx + (lane >> 2) * nxy;
      unsafeAtomicAdd(&S.grad[(size_t)c + off], (double)val);
    }
    pend &= ~__ballot(mine);
  }
}

// Merge one sample's contributions (lanes with act) into the accumulators.
__device__ __forceinline__ void accumulate(const SceneDev& S, Accum& A, bool act, int cell, const float ct[8],
                                           int lane) {
  const bool change = act && cell != A.cell;
  const bool out = change && A.cell >= 0;
  if (__ballot(out)) flush(S, A, out, lane);
  if (change) {
#pragma unroll
    for (int k = 0; k < 8; ++k) A.acc[k] = 0.0f;
    A.cell = cell;
  }
  if (act) {
#pragma unroll
    for (int k = 0; k < 8; ++k) A.acc[k] += ct[k];
  }
}

template <int DT>
__device__ __forceinline__ void load_ckpt(const SceneDev& S, int r, int slot, State& st) {
  const float* ck = S.ckpt + (size_t)r + (size_t)slot * 6 * (size_t)S.ckpt_pad;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    st.d[a] = ck[(size_t)a * S.ckpt_pad];
    st.e[a] = ck[(size_t)(3 + a) * S.ckpt_pad];
  }
}

__device__ __forceinline__ void locate_state(const SceneDev& S, const RayBase& B, const State& st, Cell& C) {
  float sm[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) sm[a] = small_part(B, a, st.jf, st.d[a]);
  locate3(S, st.bh, sm, C);
}

// Adjoint of the wall step from the final state: lambda_X = lu e_u + lv e_v;
// lambda_x = lambda_X - n (v . lambda_X)/(v . n), lambda_v = s lambda_x (metres), then
// to grid units (times the voxel size).
__device__ __forceinline__ void wall_adjoint(const SceneDev& S, const RayBase& B, const State& st, float lu, float lv,
                                             float r[3], float t[3]) {
  float dX[3], s = 0.0f;
  wall_deflection(S, B, st, dX, &s);
  float v[3], lX[3], vn = 0.0f, vl = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    v[a] = B.V[a] + st.e[a] * S.vox[a];
    lX[a] = lu * S.wall_u_f[a] + lv * S.wall_v_f[a];
    vn += v[a] * S.wall_n_f[a];
    vl += v[a] * lX[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float lx = lX[a] - S.wall_n_f[a] * (vl / vn);
    r[a] = lx * S.vox[a];
    t[a] = s * lx * S.vox[a];
  }
}

template <int DT, int KS>
__device__ __forceinline__ void adjoint_tile(const SceneDev& S, int tile, int lane) {
  int r = 0, pix = 0;
  const bool valid = tile_ray(S, tile, lane, r, pix);
  int n = 0;
  float lu = 0.0f, lv = 0.0f;
  bool active = false;
  Ray R;
  RayBase B;
  Cell C0;
  if (valid) {
    n = S.n_steps[r];
    const unsigned char st = S.status[r];
    lu = S.adj_dL_duv[2 * (size_t)r];
    lv = S.adj_dL_duv[2 * (size_t)r + 1];
    active = n > 0 && !(st & (RAY_NO_WALL_HIT | RAY_NONFINITE | RAY_MISSED_BOX)) && !(lu == 0.0f && lv == 0.0f);
    if (active) {
      setup_ray(S, pix, R);
      make_base<DT>(S, R, B, C0);
    }
  }
  const int K = S.ckpt_k;
  const int m_chunks = K / KS;
  const int nseg_lane = active ? (n + K - 1) / K : 0;
  const int nseg = wave_max_nonneg(nseg_lane);

  Accum A;
#pragma unroll
  for (int k = 0; k < 8; ++k) A.acc[k] = 0.0f;
  A.cell = -1;
  float rb[3] = {0.0f, 0.0f, 0.0f}, tb[3] = {0.0f, 0.0f, 0.0f};  // dL/dd, dL/de (grid units)
  const float h = S.hf, h_2 = S.h_2, h_6 = S.h_6, h2_8 = S.h2_8, h2_2 = S.h2_2;

  for (int seg = nseg - 1; seg >= 0; --seg) {
    for (int ch = m_chunks - 1; ch >= 0; --ch) {
      const int c0 = seg * K + ch * KS;  // first step of the chunk
      const bool lane_chunk = active && c0 < n;
      float sd[KS][3], se[KS][3];
      State st;
      if (lane_chunk) {
        state_at_step(B, seg * K, st);
        if (seg == 0) {
#pragma unroll
          for (int a = 0; a < 3; ++a) { st.d[a] = 0.0f; st.e[a] = 0.0f; }
        } else {
          load_ckpt<DT>(S, r, seg - 1, st);
        }
        Cell C;
        locate_state(S, B, st, C);
        for (int i = 0; i < ch * KS; ++i) sharma_step<DT>(S, B, st, C);  // to the chunk start
#pragma unroll
        for (int i = 0; i < KS; ++i) {
#pragma unroll
          for (int a = 0; a < 3; ++a) { sd[i][a] = st.d[a]; se[i][a] = st.e[a]; }
          if (c0 + i < n) sharma_step<DT>(S, B, st, C);
        }
        if (c0 <= n - 1 && n - 1 < c0 + KS) wall_adjoint(S, B, st, lu, lv, rb, tb);
      }
      // reverse the chunk's steps
#pragma unroll
      for (int i = KS - 1; i >= 0; --i) {
        const bool act = lane_chunk && (c0 + i < n);
        int cellA = 0, cellB = 0, cellC = 0;
        float cA[8], cB[8], cC[8];
        if (act) {
          State s;
          s.jf = (float)(2 * (c0 + i));
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            s.d[a] = sd[i][a];
            s.e[a] = se[i][a];
            s.bh[a] = fmaf(s.jf, B.g2hi[a], B.U0hi[a]);
          }
          // recompute the step's three samples (same arithmetic as the forward)
          SampleRev S1, S2, S3;
          float K1[3], K2[3], K3[3], bh2[3], bh3[3], sm[3];
          Cell C;
          locate_state(S, B, s, C);
          sample_rev<DT>(S, C, S1, K1);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            bh2[a] = s.bh[a] + B.g2hi[a];
            float dev = s.d[a] + fmaf(h_2, s.e[a], h2_8 * K1[a]);
            sm[a] = small_part(B, a, s.jf + 1.0f, dev);
          }
          locate3(S, bh2, sm, C);
          sample_rev<DT>(S, C, S2, K2);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            bh3[a] = bh2[a] + B.g2hi[a];
            float dev = s.d[a] + fmaf(h, s.e[a], h2_2 * K2[a]);
            sm[a] = small_part(B, a, s.jf + 2.0f, dev);
          }
          locate3(S, bh3, sm, C);
          sample_rev<DT>(S, C, S3, K3);
          // stage adjoints from (rb, tb) = dL/d(d', e')
          float ab[3], bb[3], v[3], p3[3], p2[3], p1[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            ab[a] = fmaf(h_6, rb[a], tb[a] * (1.0f / 6.0f));
            bb[a] = fmaf(h * (1.0f / 3.0f), rb[a], tb[a] * (2.0f / 3.0f));
            v[a] = h * (tb[a] * (1.0f / 6.0f));
          }
          force_rev(S, S3, v, p3, cC);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            bb[a] = fmaf(h_2, p3[a], bb[a]);
            v[a] = h * bb[a];
          }
          force_rev(S, S2, v, p2, cB);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            ab[a] = fmaf(h * 0.125f, p2[a], ab[a]);
            v[a] = h * ab[a];
          }
          force_rev(S, S1, v, p1, cA);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            float rn = rb[a] + p3[a] + p2[a] + p1[a];
            float tn = fmaf(h, rb[a], tb[a]) + fmaf(h, p3[a], h_2 * p2[a]);
            rb[a] = rn;
            tb[a] = tn;
          }
          cellC = voxel_of(S, S3.C);
          cellB = voxel_of(S, S2.C);
          cellA = voxel_of(S, S1.C);
        }
        accumulate(S, A, act, cellC, cC, lane);
        accumulate(S, A, act, cellB, cB, lane);
        accumulate(S, A, act, cellA, cA, lane);
      }
    }
  }
  // initial condition v0 = (1 + delta(x0)) dir: dL/d delta_c += w_c(x0) sum_a tb_a dir_a / voxel_a
  int cell0 = 0;
  float c0v[8];
  if (active) {
    float kap = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) kap = fmaf(tb[a], dd_to_f(R.dir[a]) * dd_to_f(S.inv_vox[a]), kap);
    const float X[2] = {1.0f - C0.f[0], C0.f[0]}, Y[2] = {1.0f - C0.f[1], C0.f[1]}, Z[2] = {1.0f - C0.f[2], C0.f[2]};
#pragma unroll
    for (int k = 0; k < 8; ++k) c0v[k] = kap * (X[k & 1] * Y[(k >> 1) & 1] * Z[k >> 2]);
    cell0 = voxel_of(S, C0);
  }
  accumulate(S, A, active, cell0, c0v, lane);
  flush(S, A, A.cell >= 0, lane);
}

template <int DT, int KS>
__global__ __launch_bounds__(256) void k_trace_adj(const SceneDev* __restrict__ scenes, int n_scenes, int total_tiles,
                                                   int wpb, int nblocks) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gtile = xcd_remap(blockIdx.x, nblocks) * wpb + wave;
  if (gtile >= total_tiles) return;  // whole wavefront
  const int si = find_scene(scenes, n_scenes, gtile);
  const SceneDev& S = scenes[si];
  adjoint_tile<DT, KS>(S, gtile - S.tile_begin, lane);
}

template <int DT, int KS>
__global__ __launch_bounds__(256) void k_trace_adj_persistent(const SceneDev* __restrict__ scenes, int n_scenes,
                                                              int total_tiles, unsigned int* __restrict__ queues) {
  const int lane = threadIdx.x & 63;
  const int xcd = blockIdx.x & 7;
  for (int q = 0; q < 8; ++q) {
    const int qx = (xcd + q) & 7;
    const int q_begin = (int)(((long long)total_tiles * qx) >> 3);
    const int q_end = (int)(((long long)total_tiles * (qx + 1)) >> 3);
    while (true) {
      int t = 0;
      if (lane == 0) t = (int)atomicAdd(&queues[8 + qx], 1u);
      t = __shfl(t, 0) + q_begin;
      if (t >= q_end) break;
      const int si = find_scene(scenes, n_scenes, t);
      const SceneDev& S = scenes[si];
      adjoint_tile<DT, KS>(S, t - S.tile_begin, lane);
    }
  }
}

template <int DT, int KS>
static hipError_t launch_adj_t(const LaunchPlan& P, hipStream_t stream) {
  if (P.persistent) {
    hipLaunchKernelGGL((k_trace_adj_persistent<DT, KS>), dim3(P.persistent_blocks), dim3(64 * P.wpb), 0, stream,
                       P.scenes, P.n_scenes, P.total_tiles, P.queues);
  } else {
    int nblocks = (P.total_tiles + P.wpb - 1) / P.wpb;
    hipLaunchKernelGGL((k_trace_adj<DT, KS>), dim3(nblocks), dim3(64 * P.wpb), 0, stream, P.scenes, P.n_scenes,
                       P.total_tiles, P.wpb, nblocks);
  }
  return hipGetLastError();
}

hipError_t launch_trace_adj(const LaunchPlan& P, hipStream_t stream) {
  if (P.total_tiles == 0) return hipSuccess;
  // register chunk: 8 states for stride 8, else 16 (strides 16, 32, ... replay in chunks)
  const bool k8 = (P.ckpt_k == 8);
  switch (P.dtype) {
    case DT_F32: return k8 ? launch_adj_t<DT_F32, 8>(P, stream) : launch_adj_t<DT_F32, 16>(P, stream);
    case DT_F16: return k8 ? launch_adj_t<DT_F16, 8>(P, stream) : launch_adj_t<DT_F16, 16>(P, stream);
    default: return k8 ? launch_adj_t<DT_BF16, 8>(P, stream) : launch_adj_t<DT_BF16, 16>(P, stream);
  }
}

}  // namespace rbos
