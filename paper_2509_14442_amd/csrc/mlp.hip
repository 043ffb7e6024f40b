// mlp.hip -- the network field of Sec. 2.D on the matrix cores: (T_nd, p, u) = MLP(xhat)
// with tanh hidden layers of 64 units, its parameter gradient for any loss given per
// point as dL/d(outputs), and the chain from dL/d(eta - 1) on the voxel grid to
// dL/dT_nd (eta - 1 = rho0 G T0 / T, T = T0 + (T_in - T0) T_nd).
//
// The 64 x 64 layers are v_mfma_f32_32x32x2f32 products (FP32 inputs and accumulation):
// one wavefront computes a 32-point x 64-unit tile, its lanes holding the tile's inputs
// along K in two halves (lane half h supplies k = 32h + s at step s), with the bias and
// tanh applied to the accumulators before the store. The parameter gradient, a sum over
// points of outer products, runs on the same instruction with the points as K; each
// block reduces a fixed range of points and a second kernel sums the blocks in order,
// so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "mlp_launch.hpp"

namespace rbos {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row of the 32 x 32 accumulator held in register r of a lane in half h (its column is
// the lane index mod 32).
__device__ __forceinline__ int acc_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// normalised input of point p
__device__ __forceinline__ void xhat(const MlpDev& M, long long p, float x[3]) {
  if (M.points) {
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = fmaf(M.points[3 * p + a], M.xs[a], M.xo[a]);
  } else {
    const long long q = p / M.nx;
    const int i = (int)(p - q * M.nx);
    const int j = (int)(q % M.ny);
    const int k = (int)(q / M.ny);
    x[0] = (float)(2 * i + 1) / (float)M.nx - 1.0f;
    x[1] = (float)(2 * j + 1) / (float)M.ny - 1.0f;
    x[2] = (float)(2 * k + 1) / (float)M.nz - 1.0f;
  }
}

// a_1 = tanh(xhat W_0 + b_0): one thread per (point, unit)
__global__ __launch_bounds__(256) void k_mlp_first(MlpDev M, float* __restrict__ a1) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long p = idx >> 6;
  const int j = (int)(idx & 63);
  if (p >= M.n) return;
  float x[3];
  xhat(M, p, x);
  const float* W = M.params + M.off_w[0];
  float z = M.params[M.off_b[0] + j];
#pragma unroll
  for (int a = 0; a < 3; ++a) z = fmaf(x[a], W[a * MLP_WIDTH + j], z);
  a1[p * MLP_WIDTH + j] = tanhf(z);
}

// One 32-row tile of C = A B (A [n][64], B [64][64] row-major, C [n][64]) per wavefront,
// then the epilogue: TANH: C = tanh(C + bias); DTANH: C *= 1 - a^2 (a [n][64]).
template <bool DTANH>
__global__ __launch_bounds__(256) void k_mlp_dense(long long n, const float* __restrict__ A, const float* __restrict__ B,
                                                   const float* __restrict__ bias, const float* __restrict__ act,
                                                   float* __restrict__ C) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long row0 = ((long long)blockIdx.x * 4 + wave) * 32;
  if (row0 >= n) return;  // whole wavefronts only: every lane takes part in the products
  const int c = lane & 31, h = lane >> 5;
  const long long row = row0 + c;
  float a[32];
  if (row < n) {
    const f32x4* pa = reinterpret_cast<const f32x4*>(A + row * MLP_WIDTH + 32 * h);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const f32x4 v = pa[q];
      a[4 * q] = v.x; a[4 * q + 1] = v.y; a[4 * q + 2] = v.z; a[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int s = 0; s < 32; ++s) a[s] = 0.0f;
  }
  f32x16 acc0 = {}, acc1 = {};
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    const float* pb = B + (32 * h + s) * MLP_WIDTH;
    acc0 = mfma32(a[s], pb[c], acc0);
    acc1 = mfma32(a[s], pb[32 + c], acc1);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const f32x16& acc = t == 0 ? acc0 : acc1;
    const int col = 32 * t + c;
    const float bc = DTANH ? 0.0f : bias[col];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const long long rr = row0 + acc_row(r, h);
      if (rr < n) {
        float v;
        if constexpr (DTANH) {
          const float y = act[rr * MLP_WIDTH + col];
          v = acc[r] * (1.0f - y * y);
        } else {
          v = tanhf(acc[r] + bc);
        }
        C[rr * MLP_WIDTH + col] = v;
      }
    }
  }
}

// out = a_D W_D + b_D (and T = T0 + dT out_0): one thread per (point, output), 8 slots
// per point
__global__ __launch_bounds__(256) void k_mlp_out(MlpDev M, const float* __restrict__ aD, float* __restrict__ out,
                                                 float* __restrict__ T, float T0, float dT) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long p = idx >> 3;
  const int o = (int)(idx & 7);
  if (p >= M.n || o >= MLP_OUT) return;
  const float* W = M.params + M.off_w[M.depth];
  const float* a = aD + p * MLP_WIDTH;
  float z = M.params[M.off_b[M.depth] + o];
  for (int k = 0; k < MLP_WIDTH; ++k) z = fmaf(a[k], W[k * MLP_OUT + o], z);
  if (out) out[p * MLP_OUT + o] = z;
  if (T && o == 0) T[p] = fmaf(dT, z, T0);
}

// delta_D = (dL/dout W_D^T) (1 - a_D^2): one thread per (point, unit)
__global__ __launch_bounds__(256) void k_mlp_delta_out(MlpDev M, const float* __restrict__ dL,
                                                       const float* __restrict__ aD, float* __restrict__ delta) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long p = idx >> 6;
  const int j = (int)(idx & 63);
  if (p >= M.n) return;
  const float* W = M.params + M.off_w[M.depth];
  float g = 0.0f;
#pragma unroll
  for (int o = 0; o < MLP_OUT; ++o) g = fmaf(dL[p * MLP_OUT + o], W[j * MLP_OUT + o], g);
  const float y = aD[p * MLP_WIDTH + j];
  delta[p * MLP_WIDTH + j] = g * (1.0f - y * y);
}

// WT_l = W_l^T for the hidden layers l = 1 .. depth - 1
__global__ __launch_bounds__(256) void k_mlp_transpose(MlpDev M, float* __restrict__ wt) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int l = 1 + idx / (MLP_WIDTH * MLP_WIDTH);
  if (l >= M.depth) return;
  const int e = idx % (MLP_WIDTH * MLP_WIDTH), k = e / MLP_WIDTH, j = e % MLP_WIDTH;
  wt[(l - 1) * MLP_WIDTH * MLP_WIDTH + j * MLP_WIDTH + k] = M.params[M.off_w[l] + k * MLP_WIDTH + j];
}

// Partial parameter gradient of one layer over this block's points:
// P[m][j] = sum_i A[i][m] B[i][j] (m < 64, j < 64) and P[4096 + j] = sum_i B[i][j].
// A: the layer's input (XHAT: the normalised positions, 3 columns; else a [n][64]);
// B: the gradient at its output, ldb columns of which nb are used. One wavefront per
// block, the points along K in 64-point chunks.
template <bool XHAT>
__global__ __launch_bounds__(64) void k_mlp_wgrad(MlpDev M, const float* __restrict__ A, const float* __restrict__ B,
                                                  int ldb, int nb, float* __restrict__ partial,
                                                  long long rows_per_block) {
  constexpr int MT = XHAT ? 1 : 2;
  const int lane = threadIdx.x, c = lane & 31, h = lane >> 5;
  const long long r0 = (long long)blockIdx.x * rows_per_block;
  const long long r1 = r0 + rows_per_block < M.n ? r0 + rows_per_block : M.n;
  f32x16 acc[MT][2];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) acc[mt][0] = acc[mt][1] = f32x16{};
  float bsum[2] = {0.0f, 0.0f};
  for (long long base = r0; base < r1; base += 64) {
#pragma unroll 4
    for (int s = 0; s < 32; ++s) {
      const long long row = base + 32 * h + s;
      const bool ok = row < r1;
      float a[MT], b[2];
      if constexpr (XHAT) {
        float x[3] = {0.0f, 0.0f, 0.0f};
        if (ok) xhat(M, row, x);
        a[0] = c < 3 ? x[c] : 0.0f;
      } else {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = ok ? A[row * MLP_WIDTH + 32 * mt + c] : 0.0f;
      }
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int col = 32 * nt + c;
        b[nt] = (ok && col < nb) ? B[row * ldb + col] : 0.0f;
        bsum[nt] += b[nt];
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        acc[mt][0] = mfma32(a[mt], b[0], acc[mt][0]);
        if (nb > 32) acc[mt][1] = mfma32(a[mt], b[1], acc[mt][1]);
      }
    }
  }
  float* P = partial + (long long)blockIdx.x * MLP_PART;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      if (nt == 1 && nb <= 32) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) P[(32 * mt + acc_row(r, h)) * MLP_WIDTH + 32 * nt + c] = acc[mt][nt][r];
    }
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const float other = __shfl_xor(bsum[nt], 32);
    if (h == 0) P[MLP_WIDTH * MLP_WIDTH + 32 * nt + c] = bsum[nt] + other;
  }
}

// dparams[layer] += sum over blocks (in block order) of the partials: W [fi][fo], b [fo]
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, int nblk, int fi, int fo,
                                                    float* __restrict__ dW, float* __restrict__ db) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= fi * fo + fo) return;
  const int src = e < fi * fo ? (e / fo) * MLP_WIDTH + e % fo : MLP_WIDTH * MLP_WIDTH + (e - fi * fo);
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += partial[(long long)b * MLP_PART + src];
  if (e < fi * fo) dW[e] += s;
  else db[e - fi * fo] += s;
}

__global__ __launch_bounds__(256) void k_mlp_bos_seed(long long n, const float* __restrict__ T,
                                                      const double* __restrict__ grad, double k, float* __restrict__ dL) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const double t = (double)T[p];
  dL[p * MLP_OUT] = (float)(grad[p] * (k / (t * t)));
#pragma unroll
  for (int o = 1; o < MLP_OUT; ++o) dL[p * MLP_OUT + o] = 0.0f;
}

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int blocks_for(long long threads) { return (int)((threads + 255) / 256); }

}  // namespace

size_t mlp_work_bytes(int depth, long long n) {
  long long nblk = (n + 63) / 64;
  if (nblk > 1024) nblk = 1024;
  if (nblk < 1) nblk = 1;
  size_t b = 0;
  b += al256(sizeof(float) * (size_t)depth * (size_t)n * MLP_WIDTH);
  b += 2 * al256(sizeof(float) * (size_t)n * MLP_WIDTH);
  b += al256(sizeof(float) * (size_t)(depth > 1 ? depth - 1 : 1) * MLP_WIDTH * MLP_WIDTH);
  b += al256(sizeof(float) * (size_t)(depth + 1) * (size_t)nblk * MLP_PART);
  return b;
}

void mlp_work_carve(void* ws, int depth, long long n, MlpWork& w) {
  long long nblk = (n + 63) / 64;
  if (nblk > 1024) nblk = 1024;
  if (nblk < 1) nblk = 1;
  w.nblk = (int)nblk;
  long long rows = (n + nblk - 1) / nblk;
  w.rows_per_block = (rows + 63) / 64 * 64;
  unsigned char* p = static_cast<unsigned char*>(ws);
  w.act = reinterpret_cast<float*>(p);
  p += al256(sizeof(float) * (size_t)depth * (size_t)n * MLP_WIDTH);
  w.delta[0] = reinterpret_cast<float*>(p);
  p += al256(sizeof(float) * (size_t)n * MLP_WIDTH);
  w.delta[1] = reinterpret_cast<float*>(p);
  p += al256(sizeof(float) * (size_t)n * MLP_WIDTH);
  w.wt = reinterpret_cast<float*>(p);
  p += al256(sizeof(float) * (size_t)(depth > 1 ? depth - 1 : 1) * MLP_WIDTH * MLP_WIDTH);
  w.partial = reinterpret_cast<float*>(p);
}

hipError_t launch_mlp_forward(const MlpDev& M, const MlpWork& w, float* out, float* T, float T0, float dT,
                              hipStream_t stream) {
  if (M.n == 0) return hipSuccess;
  const long long n = M.n;
  hipLaunchKernelGGL(k_mlp_first, dim3(blocks_for(n * MLP_WIDTH)), dim3(256), 0, stream, M, w.act);
  for (int l = 1; l < M.depth; ++l) {
    const float* ain = w.act + (size_t)(l - 1) * n * MLP_WIDTH;
    float* aout = w.act + (size_t)l * n * MLP_WIDTH;
    hipLaunchKernelGGL((k_mlp_dense<false>), dim3((unsigned)((n + 127) / 128)), dim3(256), 0, stream, n, ain,
                       M.params + M.off_w[l], M.params + M.off_b[l], nullptr, aout);
  }
  if (out || T) {
    const float* aD = w.act + (size_t)(M.depth - 1) * n * MLP_WIDTH;
    hipLaunchKernelGGL(k_mlp_out, dim3(blocks_for(n * 8)), dim3(256), 0, stream, M, aD, out, T, T0, dT);
  }
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const MlpDev& M, const MlpWork& w, const float* dL_dout, float* dparams,
                               hipStream_t stream) {
  if (M.n == 0) return hipSuccess;
  const long long n = M.n;
  const int D = M.depth;
  auto act = [&](int l) { return w.act + (size_t)(l - 1) * n * MLP_WIDTH; };  // a_l, l = 1 .. D
  auto part = [&](int l) { return w.partial + (size_t)l * w.nblk * MLP_PART; };
  if (D > 1)
    hipLaunchKernelGGL(k_mlp_transpose, dim3(blocks_for((long long)(D - 1) * MLP_WIDTH * MLP_WIDTH)), dim3(256), 0,
                       stream, M, w.wt);
  // output layer: dW_D = a_D^T dL, db_D = sum dL; delta_D = (dL W_D^T)(1 - a_D^2)
  hipLaunchKernelGGL((k_mlp_wgrad<false>), dim3(w.nblk), dim3(64), 0, stream, M, act(D), dL_dout, MLP_OUT, MLP_OUT,
                     part(D), w.rows_per_block);
  hipLaunchKernelGGL(k_mlp_delta_out, dim3(blocks_for(n * MLP_WIDTH)), dim3(256), 0, stream, M, dL_dout, act(D),
                     w.delta[0]);
  int cur = 0;
  for (int l = D - 1; l >= 1; --l) {
    // dW_l = a_l^T delta_{l+1}; delta_l = (delta_{l+1} W_l^T)(1 - a_l^2)
    hipLaunchKernelGGL((k_mlp_wgrad<false>), dim3(w.nblk), dim3(64), 0, stream, M, act(l), w.delta[cur], MLP_WIDTH,
                       MLP_WIDTH, part(l), w.rows_per_block);
    hipLaunchKernelGGL((k_mlp_dense<true>), dim3((unsigned)((n + 127) / 128)), dim3(256), 0, stream, n, w.delta[cur],
                       w.wt + (size_t)(l - 1) * MLP_WIDTH * MLP_WIDTH, nullptr, act(l), w.delta[cur ^ 1]);
    cur ^= 1;
  }
  hipLaunchKernelGGL((k_mlp_wgrad<true>), dim3(w.nblk), dim3(64), 0, stream, M, nullptr, w.delta[cur], MLP_WIDTH,
                     MLP_WIDTH, part(0), w.rows_per_block);
  for (int l = 0; l <= D; ++l) {
    const int fi = l == 0 ? 3 : MLP_WIDTH, fo = l == D ? MLP_OUT : MLP_WIDTH;
    hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks_for(fi * fo + fo)), dim3(256), 0, stream, part(l), w.nblk, fi, fo,
                       dparams + M.off_w[l], dparams + M.off_b[l]);
  }
  return hipGetLastError();
}

hipError_t launch_mlp_bos_seed(long long n, const float* T, const double* grad_delta, double rho0G, double T0,
                               double dT, float* dL_dout, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const double k = -rho0G * T0 * dT;
  hipLaunchKernelGGL(k_mlp_bos_seed, dim3(blocks_for(n)), dim3(256), 0, stream, n, T, grad_delta, k, dL_dout);
  return hipGetLastError();
}

}  // namespace rbos
