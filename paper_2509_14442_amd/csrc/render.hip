// render.hip -- Sec. 2.C / 2.D: wall luminance at each traced hit (printed texture or
// pinhole projector, bilinear, zero outside; optionally times the radiometric weight),
// pixel values as the mean of their rays (Eq. 2), residual against the measured image,
// L_BOS = sum_j r_j^2 (deterministic: per-block partials, then one fixed-order pass per
// scene) and per ray dL_BOS/d(u, v) = 2 r_j dI_j/d(u, v).
#include "rbos_device.hpp"
#include "rbos_launch.hpp"

namespace rbos {

// floor / fraction of a double-float texel coordinate
__device__ __forceinline__ void texel_split(df a, int& i, float& f) {
  float fl = floorf(a.hi);
  float ff = (a.hi - fl) + a.lo;
  if (ff < 0.0f) { ff += 1.0f; fl -= 1.0f; }
  else if (ff >= 1.0f) { ff -= 1.0f; fl += 1.0f; }
  i = (int)fl;
  f = ff;
}

__device__ __forceinline__ float texel(const SceneDev& S, int row, int col, bool& inside) {
  if (row < 0 || row >= S.pat_h || col < 0 || col >= S.pat_w) return 0.0f;
  inside = true;
  return gld(S.pattern + (size_t)row * S.pat_w + col);
}

// bilinear lookup at texel coordinates (a, b) = (column, row), texel centres at integers
__device__ __forceinline__ float bilinear(const SceneDev& S, df a, df b, float& dIda, float& dIdb, bool& off) {
  int a0, b0;
  float fa, fb;
  texel_split(a, a0, fa);
  texel_split(b, b0, fb);
  if (!isfinite(fa) || !isfinite(fb) || a.hi < -2.0f || b.hi < -2.0f || a.hi > (float)S.pat_w + 2.0f ||
      b.hi > (float)S.pat_h + 2.0f) {
    off = true;
    dIda = dIdb = 0.0f;
    return 0.0f;
  }
  bool inside = false;
  float t00 = texel(S, b0, a0, inside), t01 = texel(S, b0, a0 + 1, inside);
  float t10 = texel(S, b0 + 1, a0, inside), t11 = texel(S, b0 + 1, a0 + 1, inside);
  off = !inside;
  dIda = (1.0f - fb) * (t01 - t00) + fb * (t11 - t10);
  dIdb = (1.0f - fa) * (t10 - t00) + fa * (t11 - t01);
  return (1.0f - fb) * ((1.0f - fa) * t00 + fa * t01) + fb * ((1.0f - fa) * t10 + fa * t11);
}

// Luminance at wall coordinates (u, v) and dI/d(u, v).
__device__ __forceinline__ float wall_luminance(const SceneDev& S, df u, df v, float dI[2], bool& off) {
  float dIda, dIdb;
  if (S.wall_mode == 0) {  // printed texture centred on the wall origin
    df a = dd_add_f(dd_mul(dd_add(u, S.pat_half_u), S.pat_inv_tu), -0.5f);
    df b = dd_add_f(dd_mul(dd_sub(S.pat_half_v, v), S.pat_inv_tv), -0.5f);
    float I = bilinear(S, a, b, dIda, dIdb, off);
    dI[0] = dIda * dd_to_f(S.pat_inv_tu);
    dI[1] = -dIdb * dd_to_f(S.pat_inv_tv);
    return I;
  }
  // pinhole projector: the wall point is lit through the projector pixel on its line
  df Y[3];
  for (int k = 0; k < 3; ++k)
    Y[k] = dd_sub(dd_add(S.wall_org[k], dd_add(dd_mul(u, S.wall_u[k]), dd_mul(v, S.wall_v[k]))), S.proj_pos[k]);
  df z = dd_dot3(Y, S.proj_fwd);
  if (!(z.hi > 0.0f)) {
    off = true;
    dI[0] = dI[1] = 0.0f;
    return 0.0f;
  }
  df yr = dd_dot3(Y, S.proj_right), yu = dd_dot3(Y, S.proj_up);
  df xp = dd_div(dd_mul(yr, S.proj_inv_tx), z);
  df yp = dd_div(dd_mul(yu, S.proj_inv_ty), z);
  float hw = 0.5f * (float)S.pat_w, hh = 0.5f * (float)S.pat_h;
  df a = dd_add_f(dd_mul_f(dd_add_f(xp, 1.0f), hw), -0.5f);
  df b = dd_add_f(dd_mul_f(dd_sub(df{1.0f, 0.0f}, yp), hh), -0.5f);
  float I = bilinear(S, a, b, dIda, dIdb, off);
  float zf = dd_to_f(z), xr = dd_to_f(yr) / zf, xu = dd_to_f(yu) / zf;
  float itx = dd_to_f(S.proj_inv_tx), ity = dd_to_f(S.proj_inv_ty);
  float g[3];
  for (int k = 0; k < 3; ++k) {
    float f = dd_to_f(S.proj_fwd[k]);
    float dxp = itx * (dd_to_f(S.proj_right[k]) - xr * f) / zf;
    float dyp = ity * (dd_to_f(S.proj_up[k]) - xu * f) / zf;
    g[k] = dIda * hw * dxp - dIdb * hh * dyp;
  }
  dI[0] = g[0] * S.wall_u_f[0] + g[1] * S.wall_u_f[1] + g[2] * S.wall_u_f[2];
  dI[1] = g[0] * S.wall_v_f[0] + g[1] * S.wall_v_f[1] + g[2] * S.wall_v_f[2];
  return I;
}

// Radiance of ray r (its sample of Eq. 2) and its derivatives w.r.t. (u, v) and, with the
// radiometric weight w = |<n_w, d>| / |X_w - c|, w.r.t. the unit direction d at the wall.
// Sets RBOS_RAY_OFF_PATTERN in the status.
__device__ __forceinline__ float ray_radiance(const SceneDev& S, int r, int pix, int smp, float dI[2], float dId[3]) {
  dI[0] = dI[1] = 0.0f;
  dId[0] = dId[1] = dId[2] = 0.0f;
  const unsigned char st = gld(S.status + r);
  if (st & (RAY_NO_WALL_HIT | RAY_NONFINITE)) return 0.0f;
  df dir[3], uv0[2];
  camera_ray(S, pix, smp, dir);
  bool off = false;
  float I = 0.0f;
  df u = {0.0f, 0.0f}, v = {0.0f, 0.0f};
  if (wall_hit_straight(S, dir, uv0)) {
    u = dd_add_f(uv0[0], gld(S.duv + 2 * (size_t)r));
    v = dd_add_f(uv0[1], gld(S.duv + 2 * (size_t)r + 1));
    I = wall_luminance(S, u, v, dI, off);
  } else {
    off = true;
  }
  if (off) gst(S.status + r, (unsigned char)(st | RAY_OFF_PATTERN));
  if (S.radiometry && !off) {
    float R[3], d[3], R2 = 0.0f, c = 0.0f;
    const float uf = dd_to_f(u), vf = dd_to_f(v);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R[k] = (S.wall_org_f[k] - dd_to_f(S.cam_pos[k])) + uf * S.wall_u_f[k] + vf * S.wall_v_f[k];
      d[k] = gld(S.wall_dir + 3 * (size_t)r + k);
      R2 += R[k] * R[k];
      c += S.wall_n_f[k] * d[k];
    }
    const float inv_dist = 1.0f / sqrtf(R2), ac = fabsf(c), w = ac * inv_dist;
    const float kk = -w * inv_dist * inv_dist;  // dw/dR = -|c| R / |R|^3
    float Ru = 0.0f, Rv = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Ru += R[k] * S.wall_u_f[k];
      Rv += R[k] * S.wall_v_f[k];
    }
    dI[0] = dI[0] * w + I * (kk * Ru);
    dI[1] = dI[1] * w + I * (kk * Rv);
    const float sg = c < 0.0f ? -inv_dist : inv_dist;
#pragma unroll
    for (int k = 0; k < 3; ++k) dId[k] = I * (sg * S.wall_n_f[k]);
    I *= w;
  }
  return I;
}

// One thread per pixel: the mean of its spp rays (Eq. 2), the residual against the
// target, and per ray dL/d(u, v) = 2 r dI_s/d(u, v) / spp (likewise dL/d(direction)).
// The per-ray derivatives are stored divided by spp on the first pass and scaled by 2 r
// once the pixel's value is known.
__global__ __launch_bounds__(256) void k_render(const SceneDev* __restrict__ scenes, int n_scenes,
                                                int total_blocks, float* __restrict__ partials) {
  __shared__ float red[4];
  const int blk = blockIdx.x;
  int si = 0;
  {
    int lo = 0, hi = n_scenes - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (scenes[mid].render_block_begin <= blk) lo = mid;
      else hi = mid - 1;
    }
    si = lo;
  }
  const SceneDev& S = scenes[si];
  const int i = (blk - S.render_block_begin) * 256 + threadIdx.x;
  float res2 = 0.0f;
  if (i < S.n_pix) {
    const int pix = S.pixel_ids ? gld(S.pixel_ids + i) : i;
    const int spp = S.spp;
    const bool grad = S.target && S.dL_duv;
    const bool grad_dir = grad && S.radiometry && S.dL_ddir;
    const float inv_spp = 1.0f / (float)spp;
    float sum = 0.0f, dI[2], dId[3];
    for (int smp = 0; smp < spp; ++smp) {
      const int r = smp * S.n_pix + i;
      sum += ray_radiance(S, r, pix, smp, dI, dId);
      if (grad) {
        gst(S.dL_duv + 2 * (size_t)r, dI[0] * inv_spp);
        gst(S.dL_duv + 2 * (size_t)r + 1, dI[1] * inv_spp);
      }
      if (grad_dir) {
#pragma unroll
        for (int k = 0; k < 3; ++k) gst(S.dL_ddir + 3 * (size_t)r + k, dId[k] * inv_spp);
      }
    }
    const float I = spp == 1 ? sum : sum * inv_spp;
    gst(S.image + i, I);
    if (S.target) {
      const float res = I - gld(S.target + i);
      res2 = res * res;
      const float g2 = 2.0f * res;
      if (grad) {
        for (int smp = 0; smp < spp; ++smp) {
          const int r = smp * S.n_pix + i;
          gst(S.dL_duv + 2 * (size_t)r, g2 * gld(S.dL_duv + 2 * (size_t)r));
          gst(S.dL_duv + 2 * (size_t)r + 1, g2 * gld(S.dL_duv + 2 * (size_t)r + 1));
          if (grad_dir) {
#pragma unroll
            for (int k = 0; k < 3; ++k) gst(S.dL_ddir + 3 * (size_t)r + k, g2 * gld(S.dL_ddir + 3 * (size_t)r + k));
          }
        }
      }
    }
  }
  if (S.target && S.loss) {
    float w = wave_sum(res2);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) partials[blk] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// one block per scene: fixed-order sum of that scene's partials
__global__ __launch_bounds__(256) void k_loss_final(const SceneDev* __restrict__ scenes,
                                                    const float* __restrict__ partials) {
  __shared__ float red[4];
  const SceneDev& S = scenes[blockIdx.x];
  if (!(S.target && S.loss)) return;
  float acc = 0.0f;
  for (int i = threadIdx.x; i < S.render_blocks; i += 256) acc += partials[S.render_block_begin + i];
  float w = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) gst(S.loss, (red[0] + red[1]) + (red[2] + red[3]));
}

hipError_t launch_render(const LaunchPlan& P, hipStream_t stream) {
  if (P.total_render_blocks > 0) {
    hipLaunchKernelGGL(k_render, dim3(P.total_render_blocks), dim3(256), 0, stream, P.scenes, P.n_scenes,
                       P.total_render_blocks, P.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_loss_final, dim3(P.n_scenes), dim3(256), 0, stream, P.scenes, P.partials);
  return hipGetLastError();
}

}  // namespace rbos
