// mlp.hip -- the network field of Sec. 2.D on the matrix cores: (T_nd, p, u) = MLP(xhat)
// with tanh hidden layers of 64 units, its parameter gradient for any loss given per
// point as dL/d(outputs), and the chain from dL/d(eta - 1) on the voxel grid to
// dL/dT_nd (eta - 1 = rho0 G T0 / T, T = T0 + (T_in - T0) T_nd).
//
// The 64 x 64 layers are v_mfma_f32_32x32x2f32 products (FP32 inputs and accumulation).
// The forward runs all layers of 32 points in one wavefront, the activations staying in
// registers between layers (k_mlp_forward_fused). The parameter gradient, a sum over
// points of outer products, runs on the same instruction with the points as K; each
// block reduces a fixed range of points and a second kernel sums the blocks in order,
// so the result does not depend on scheduling. The gradient one layer down is computed
// from the same chunk of points staged in LDS (k_mlp_wgrad with a product).
#include <hip/hip_runtime.h>

#include <atomic>

#include "mlp_launch.hpp"

namespace rbos {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// tanh x = 1 - 2 / (exp(2x) + 1), with the hardware base-2 exponential (2x / ln 2) and
// reciprocal: absolute error ~1e-7, saturating to +-1 for large |x|. The library tanhf
// costs more VALU cycles than a layer's matrix products.
__device__ __forceinline__ float tanh_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
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

// Fused forward: every layer of 32 points per wavefront, the activations kept in
// registers from layer to layer (each layer's are still written out for the backward
// pass). The hidden layers run transposed, C^T = W^T A^T (units as rows, points as
// columns), so that one layer's accumulators are the next layer's B operand as they
// stand: register r of the unit tile t in a lane of half h holds unit 32 t + acc_row(r, h)
// of point lane % 32, and step s = 16 t + r of the next product takes, in half h, that
// register with the weight W[32 t + acc_row(r, h)][unit] as the A operand (the two
// halves supply the two K values of the step). The block stages all weights in LDS once
// and its wavefronts loop over groups of 32 points.
constexpr int FUSED_PITCH = 72;  // LDS row pitch of a staged 64 x 64 weight matrix

__host__ __device__ constexpr int fused_lds_floats(int depth) {
  return (depth - 1) * MLP_WIDTH * FUSED_PITCH + depth * MLP_WIDTH + 3 * MLP_WIDTH + MLP_WIDTH * MLP_OUT + 8;
}

__global__ __launch_bounds__(256) void k_mlp_forward_fused(MlpDev M, float* __restrict__ act, float* __restrict__ xh,
                                                           float* __restrict__ out, float* __restrict__ T, float T0,
                                                           float dT) {
  extern __shared__ float lds[];
  const int D = M.depth;
  float* Wh = lds;                                         // W_1 .. W_{D-1}, rows padded
  float* bh = Wh + (D - 1) * MLP_WIDTH * FUSED_PITCH;      // b_0 .. b_{D-1}
  float* W0 = bh + D * MLP_WIDTH;                          // [3][64]
  float* WD = W0 + 3 * MLP_WIDTH;                          // [64][5]
  float* bD = WD + MLP_WIDTH * MLP_OUT;                    // [5]
  const float* P = M.params;
  for (int e = threadIdx.x; e < (D - 1) * MLP_WIDTH * MLP_WIDTH; e += 256) {
    const int l = e / (MLP_WIDTH * MLP_WIDTH), k = (e / MLP_WIDTH) % MLP_WIDTH, u = e % MLP_WIDTH;
    Wh[(l * MLP_WIDTH + k) * FUSED_PITCH + u] = P[M.off_w[l + 1] + k * MLP_WIDTH + u];
  }
  for (int e = threadIdx.x; e < D * MLP_WIDTH; e += 256) bh[e] = P[M.off_b[e / MLP_WIDTH] + e % MLP_WIDTH];
  for (int e = threadIdx.x; e < 3 * MLP_WIDTH; e += 256) W0[e] = P[M.off_w[0] + e];
  for (int e = threadIdx.x; e < MLP_WIDTH * MLP_OUT; e += 256) WD[e] = P[M.off_w[D] + e];
  if (threadIdx.x < MLP_OUT) bD[threadIdx.x] = P[M.off_b[D] + threadIdx.x];
  __syncthreads();

  const int lane = threadIdx.x & 63, c = lane & 31, h = lane >> 5;
  const long long n = M.n;
  const long long stride = (long long)gridDim.x * 4;
  for (long long g = (long long)blockIdx.x * 4 + (threadIdx.x >> 6); g * 32 < n; g += stride) {
    const long long p = g * 32 + c;
    const bool valid = p < n;
    float x[3] = {0.0f, 0.0f, 0.0f};
    if (valid) xhat(M, p, x);
    if (valid && h == 0) *reinterpret_cast<f32x4*>(xh + p * 4) = f32x4{x[0], x[1], x[2], 0.0f};
    // a[16 t + r]: unit 32 t + acc_row(r, h) of point p
    float a[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const int u = 32 * (i >> 4) + acc_row(i & 15, h);
      float z = bh[u];
#pragma unroll
      for (int d = 0; d < 3; ++d) z = fmaf(x[d], W0[d * MLP_WIDTH + u], z);
      a[i] = tanh_fast(z);
    }
    for (int l = 0; l < D; ++l) {
      if (l > 0) {
        const float* W = Wh + (l - 1) * MLP_WIDTH * FUSED_PITCH;
        f32x16 acc0 = {}, acc1 = {};
#pragma unroll
        for (int s = 0; s < 32; ++s) {
          const float* w = W + (32 * (s >> 4) + acc_row(s & 15, h)) * FUSED_PITCH;
          acc0 = mfma32(w[c], a[s], acc0);
          acc1 = mfma32(w[32 + c], a[s], acc1);
        }
        const float* b = bh + l * MLP_WIDTH;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          a[r] = tanh_fast(acc0[r] + b[acc_row(r, h)]);
          a[16 + r] = tanh_fast(acc1[r] + b[32 + acc_row(r, h)]);
        }
      }
      if (valid) {  // a_{l+1} [n][64]: units 32 t + 8 j + 4 h .. +3 are a[16 t + 4 j .. +3]
        float* dst = act + (size_t)l * (size_t)n * MLP_WIDTH + p * MLP_WIDTH + 4 * h;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          *reinterpret_cast<f32x4*>(dst + 32 * (q >> 2) + 8 * (q & 3)) =
              f32x4{a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]};
      }
    }
    if (out || T) {
      float z[MLP_OUT];
#pragma unroll
      for (int o = 0; o < MLP_OUT; ++o) z[o] = 0.0f;
#pragma unroll
      for (int i = 0; i < 32; ++i) {
        const int u = 32 * (i >> 4) + acc_row(i & 15, h);
#pragma unroll
        for (int o = 0; o < MLP_OUT; ++o) z[o] = fmaf(a[i], WD[u * MLP_OUT + o], z[o]);
      }
#pragma unroll
      for (int o = 0; o < MLP_OUT; ++o) {  // the two halves hold the point's two unit sets
        auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(z[o]), __float_as_uint(z[o]), false, false);
        z[o] = (__uint_as_float(sw[0]) + __uint_as_float(sw[1])) + bD[o];
      }
      if (valid && h == 0) {
        if (out)
#pragma unroll
          for (int o = 0; o < MLP_OUT; ++o) out[p * MLP_OUT + o] = z[o];
        if (T) T[p] = fmaf(dT, z[0], T0);
      }
    }
  }
}

// WT_l = W_l^T for the hidden layers l = 1 .. depth - 1, then the output layer's W_D^T
// (5 x 64) padded with zero rows to 64 x 64, so that its product runs like the others
__global__ __launch_bounds__(256) void k_mlp_transpose(MlpDev M, float* __restrict__ wt) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int l = 1 + idx / (MLP_WIDTH * MLP_WIDTH);
  if (l > M.depth) return;
  const int e = idx % (MLP_WIDTH * MLP_WIDTH), k = e / MLP_WIDTH, j = e % MLP_WIDTH;
  float v;
  if (l < M.depth) v = M.params[M.off_w[l] + k * MLP_WIDTH + j];
  else v = j < MLP_OUT ? M.params[M.off_w[l] + k * MLP_OUT + j] : 0.0f;
  wt[(l - 1) * MLP_WIDTH * MLP_WIDTH + j * MLP_WIDTH + k] = v;
}

// Partial parameter gradient of one layer over this block's rows:
// P[m][j] = sum_i A[i][m] B[i][j] (m < 64, j < 64) and P[4096 + j] = sum_{i < bias_rows} B[i][j].
// A: the layer's input (XHAT: the first layer's, rows i < M.n the normalised position of
// point i from xh [n][4], rows i = (1 + a) M.n + p the unit vector e_a (the input's
// derivative along a in a jet); else a [nrows][64]); B: the gradient at its output, ldb
// columns of which nb are used. Four wavefronts per block: each 64-row chunk of A and B
// is staged in LDS with coalesced loads, and wavefront (mt, nt) accumulates the 32 x 32
// tile P[32 mt ..][32 nt ..] with the rows along K.
// With PROD, the same staged chunk also gives the gradient one layer down, written to
// Cout [nrows][64]: Cout = B WT (WT = W^T as 64 x 64, zero rows past B's nb columns), times 1 - A^2
// for PROD_DTANH. Wavefront (mt, nt) computes its rows 32 mt .. and units 32 nt .., so
// A and B are read from HBM once for both products.
enum { PROD_NONE = 0, PROD_DTANH = 1, PROD_PLAIN = 2 };
template <bool XHAT, int PROD = PROD_NONE>
__global__ __launch_bounds__(256) void k_mlp_wgrad(MlpDev M, const float* __restrict__ A, const float* __restrict__ B,
                                                   int ldb, int nb, float* __restrict__ partial,
                                                   long long rows_per_block, long long nrows, long long bias_rows,
                                                   const float* __restrict__ WT = nullptr,
                                                   float* __restrict__ Cout = nullptr) {
  __shared__ float As[64 * 65];
  __shared__ float Bs[64 * 65];
  __shared__ float Ws[PROD != PROD_NONE ? 64 * 65 : 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if constexpr (PROD != PROD_NONE) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int e = t + 256 * i;
      Ws[(e >> 6) * 65 + (e & 63)] = WT[e];
    }
  }
  const int mt = wave >> 1, nt = wave & 1;
  const int c = lane & 31, h = lane >> 5;
  const long long r0 = (long long)blockIdx.x * rows_per_block;
  const long long r1 = r0 + rows_per_block < nrows ? r0 + rows_per_block : nrows;
  f32x16 acc = {};
  float bsum = 0.0f;
  // chunk elements e = t + 256 i (row e / 64, column e % 64), loaded one chunk ahead
  float av[16], bv[16];
  auto load_chunk = [&](long long base) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int e = t + 256 * i, col = e & 63;
      const long long row = base + (e >> 6);
      av[i] = 0.0f;
      bv[i] = 0.0f;
      if (row < r1) {
        if constexpr (XHAT) {
          if (col < 3) av[i] = row < M.n ? A[row * 4 + col] : (col == (int)(row / M.n) - 1 ? 1.0f : 0.0f);
        } else {
          av[i] = A[row * MLP_WIDTH + col];
        }
        if (col < nb) bv[i] = B[row * ldb + col];
      }
    }
  };
  if (r0 < r1) load_chunk(r0);
  for (long long base = r0; base < r1; base += 64) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int e = t + 256 * i;
      As[(e >> 6) * 65 + (e & 63)] = av[i];
      Bs[(e >> 6) * 65 + (e & 63)] = bv[i];
    }
    __syncthreads();
    if (base + 64 < r1) load_chunk(base + 64);  // in flight during this chunk's products
#pragma unroll 8
    for (int s = 0; s < 32; ++s) {
      const int rr = 32 * h + s;
      const float bvv = Bs[rr * 65 + 32 * nt + c];
      acc = mfma32(As[rr * 65 + 32 * mt + c], bvv, acc);
      if (mt == 0 && base + rr < bias_rows) bsum += bvv;
    }
    if constexpr (PROD != PROD_NONE) {
      // rows 32 mt + acc_row(r, h), units 32 nt + c of B WT; K = the 64 columns of B,
      // lane half h supplying k = 32 h + s at step s
      f32x16 d = {};
#pragma unroll 8
      for (int s = 0; s < 32; ++s) {
        const int k = 32 * h + s;
        d = mfma32(Bs[(32 * mt + c) * 65 + k], Ws[k * 65 + 32 * nt + c], d);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = 32 * mt + acc_row(r, h);
        if (base + rr < r1) {
          float v = d[r];
          if constexpr (PROD == PROD_DTANH) {
            const float y = As[rr * 65 + 32 * nt + c];
            v *= 1.0f - y * y;
          }
          Cout[(base + rr) * MLP_WIDTH + 32 * nt + c] = v;
        }
      }
    }
    __syncthreads();
  }
  float* P = partial + (long long)blockIdx.x * MLP_PART;
#pragma unroll
  for (int r = 0; r < 16; ++r) P[(32 * mt + acc_row(r, h)) * MLP_WIDTH + 32 * nt + c] = acc[r];
  const float other = __shfl_xor(bsum, 32);
  if (mt == 0 && h == 0) P[MLP_WIDTH * MLP_WIDTH + 32 * nt + c] = bsum + other;
}

// dparams[layer] += sum over blocks of the partials: W [fi][fo], b [fo]. A block takes 16
// elements; its 16 thread groups sum the blocks b = g, g + 16, ..., and the groups are
// added in a fixed order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, int nblk, int fi, int fo,
                                                    float* __restrict__ dW, float* __restrict__ db) {
  __shared__ float red[16][17];
  const int el = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int e = blockIdx.x * 16 + el;
  const int ne = fi * fo + fo;
  float s = 0.0f;
  if (e < ne) {
    const int src = e < fi * fo ? (e / fo) * MLP_WIDTH + e % fo : MLP_WIDTH * MLP_WIDTH + (e - fi * fo);
#pragma unroll 8
    for (int b = g; b < nblk; b += 16) s += partial[(long long)b * MLP_PART + src];
  }
  red[g][el] = s;
  __syncthreads();
  if (g == 0 && e < ne) {
    float t = red[0][el];
#pragma unroll
    for (int k = 1; k < 16; ++k) t += red[k][el];
    if (e < fi * fo) dW[e] += t;
    else db[e - fi * fo] += t;
  }
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

// ------------------------------------------------------------------------------------
// Jets for the PDE residuals: per point 7 channels of every layer's activations, the
// value (c = 0), its derivative along xhat_d (c = 1 + d) and its second derivative along
// xhat_d (c = 4 + d), stored channel-major ([7][n][64]). A linear layer maps every
// channel by the same weights (the bias enters the value only); tanh maps
// (z, z_d, z_dd) to (y, t z_d, t z_dd - 2 y t z_d^2) with y = tanh z, t = 1 - y^2.
// ------------------------------------------------------------------------------------
constexpr int JET = 7;

// first layer: the input's jet is (xhat, e_d, 0); xh [n][4] as in k_mlp_forward_fused
__global__ __launch_bounds__(256) void k_jet_first(MlpDev M, float* __restrict__ aj, float* __restrict__ zj,
                                                   float* __restrict__ xh) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long p = idx >> 6;
  const int j = (int)(idx & 63);
  const long long n = M.n;
  if (p >= n) return;
  float x[3];
  xhat(M, p, x);
  if (j < 4) xh[p * 4 + j] = j < 3 ? x[j] : 0.0f;
  const float* W = M.params + M.off_w[0];
  float z = M.params[M.off_b[0] + j];
#pragma unroll
  for (int a = 0; a < 3; ++a) z = fmaf(x[a], W[a * MLP_WIDTH + j], z);
  const float y = tanh_fast(z), t = 1.0f - y * y;
  const long long e = p * MLP_WIDTH + j, ch = n * MLP_WIDTH;
  aj[e] = y;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float zd = W[d * MLP_WIDTH + j];
    aj[(1 + d) * ch + e] = t * zd;
    aj[(4 + d) * ch + e] = -2.0f * y * t * zd * zd;
    zj[d * ch + e] = zd;
    zj[(3 + d) * ch + e] = 0.0f;
  }
}

// a hidden layer on the jets: one wavefront per 32 points and direction d = blockIdx.y
// (channels 0, 1 + d, 4 + d); the value channel is written by the d = 0 wavefronts
__global__ __launch_bounds__(256) void k_jet_dense(long long n, const float* __restrict__ aj,
                                                   const float* __restrict__ W, const float* __restrict__ bias,
                                                   float* __restrict__ aj_next, float* __restrict__ zj_next) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long row0 = ((long long)blockIdx.x * 4 + wave) * 32;
  if (row0 >= n) return;
  const int d = blockIdx.y;
  const int c = lane & 31, h = lane >> 5;
  const long long row = row0 + c, ch = n * MLP_WIDTH;
  const int chans[3] = {0, 1 + d, 4 + d};
  f32x16 acc[3][2];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    acc[q][0] = acc[q][1] = f32x16{};
    float a[32];
    if (row < n) {
      const f32x4* pa = reinterpret_cast<const f32x4*>(aj + chans[q] * ch + row * MLP_WIDTH + 32 * h);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const f32x4 v = pa[k];
        a[4 * k] = v.x; a[4 * k + 1] = v.y; a[4 * k + 2] = v.z; a[4 * k + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int s = 0; s < 32; ++s) a[s] = 0.0f;
    }
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const float* pb = W + (32 * h + s) * MLP_WIDTH;
      acc[q][0] = mfma32(a[s], pb[c], acc[q][0]);
      acc[q][1] = mfma32(a[s], pb[32 + c], acc[q][1]);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int col = 32 * t + c;
    const float bc = bias[col];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const long long rr = row0 + acc_row(r, h);
      if (rr < n) {
        const float y = tanh_fast(acc[0][t][r] + bc), tp = 1.0f - y * y;
        const float zd = acc[1][t][r], zdd = acc[2][t][r];
        const long long e = rr * MLP_WIDTH + col;
        if (d == 0) aj_next[e] = y;
        aj_next[(1 + d) * ch + e] = tp * zd;
        aj_next[(4 + d) * ch + e] = tp * zdd - 2.0f * y * tp * zd * zd;
        zj_next[d * ch + e] = zd;
        zj_next[(3 + d) * ch + e] = zdd;
      }
    }
  }
}

// output layer on the jets: oj [7][n][5]
__global__ __launch_bounds__(256) void k_jet_out(MlpDev M, const float* __restrict__ aj, float* __restrict__ oj) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long n = M.n;
  const long long q = idx >> 3;  // channel-major (c, p)
  const int o = (int)(idx & 7);
  if (q >= JET * n || o >= MLP_OUT) return;
  const int cch = (int)(q / n);
  const float* W = M.params + M.off_w[M.depth];
  const float* a = aj + q * MLP_WIDTH;
  float z = cch == 0 ? M.params[M.off_b[M.depth] + o] : 0.0f;
  for (int k = 0; k < MLP_WIDTH; ++k) z = fmaf(a[k], W[k * MLP_OUT + o], z);
  oj[q * MLP_OUT + o] = z;
}

// Boussinesq residuals (Sec. 2.D) in nondimensional coordinates from the output jets, the
// per-point loss g1 r_mass^2 + g2 |r_mom|^2 + g3 r_heat^2 (block partials) and its seed
// on every output channel. Outputs: T_nd, p, u_x, u_y, u_z; gravity along -z.
__global__ __launch_bounds__(256) void k_pde_seed(long long n, const float* __restrict__ oj, PdeConst P,
                                                  float* __restrict__ dj, float* __restrict__ res,
                                                  float* __restrict__ partials) {
  __shared__ float red[4];
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  float lp = 0.0f;
  if (p < n) {
    float v[MLP_OUT], D1[3][MLP_OUT], D2[3][MLP_OUT];
#pragma unroll
    for (int k = 0; k < MLP_OUT; ++k) {
      v[k] = oj[p * MLP_OUT + k];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        D1[d][k] = P.s[d] * oj[((1 + d) * n + p) * MLP_OUT + k];
        D2[d][k] = P.s[d] * P.s[d] * oj[((4 + d) * n + p) * MLP_OUT + k];
      }
    }
    const float T = v[0];
    const float u[3] = {v[2], v[3], v[4]};
    float rmass = 0.0f, rmom[3], rheat = 0.0f;
#pragma unroll
    for (int d = 0; d < 3; ++d) rmass += D1[d][2 + d];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float conv = 0.0f, lap = 0.0f;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        conv = fmaf(u[d], D1[d][2 + k], conv);
        lap += D2[d][2 + k];
      }
      rmom[k] = conv + D1[k][1] - lap * P.inv_re + (k == 2 ? -P.ri * T : 0.0f);
    }
    {
      float conv = 0.0f, lap = 0.0f;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        conv = fmaf(u[d], D1[d][0], conv);
        lap += D2[d][0];
      }
      rheat = conv - lap * P.inv_pe;
    }
    lp = P.g[0] * rmass * rmass + P.g[1] * (rmom[0] * rmom[0] + rmom[1] * rmom[1] + rmom[2] * rmom[2]) +
         P.g[2] * rheat * rheat;
    if (res) {
      res[p * 5] = rmass;
      res[p * 5 + 1] = rmom[0];
      res[p * 5 + 2] = rmom[1];
      res[p * 5 + 3] = rmom[2];
      res[p * 5 + 4] = rheat;
    }
    if (dj) {
      const float Rm = 2.0f * P.g[0] * rmass, Rh = 2.0f * P.g[2] * rheat;
      const float Rv[3] = {2.0f * P.g[1] * rmom[0], 2.0f * P.g[1] * rmom[1], 2.0f * P.g[1] * rmom[2]};
      // value channel
      dj[p * MLP_OUT] = -P.ri * Rv[2];
      dj[p * MLP_OUT + 1] = 0.0f;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float g = Rh * D1[d][0];
#pragma unroll
        for (int k = 0; k < 3; ++k) g = fmaf(Rv[k], D1[d][2 + k], g);
        dj[p * MLP_OUT + 2 + d] = g;
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float* g1 = dj + ((1 + d) * n + p) * MLP_OUT;
        float* g2 = dj + ((4 + d) * n + p) * MLP_OUT;
        const float sd = P.s[d], sd2 = sd * sd;
        g1[0] = Rh * u[d] * sd;
        g1[1] = Rv[d] * sd;
#pragma unroll
        for (int k = 0; k < 3; ++k) g1[2 + k] = (Rv[k] * u[d] + (k == d ? Rm : 0.0f)) * sd;
        g2[0] = -Rh * sd2 * P.inv_pe;
        g2[1] = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) g2[2 + k] = -Rv[k] * sd2 * P.inv_re;
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) lp += __shfl_xor(lp, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lp;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Reverse of tanh on the jets: from G = dL/d(a channels) [7][n][64] (OUT: from the output
// seeds dj [7][n][5] through W_D^T), the layer's y = a_0 and its pre-activation
// derivatives zj [6][n][64], writes dz = dL/d(z channels) [7][n][64].
template <bool OUT>
__global__ __launch_bounds__(256) void k_jet_act_back(MlpDev M, const float* __restrict__ G,
                                                      const float* __restrict__ aj, const float* __restrict__ zj,
                                                      float* __restrict__ dz) {
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long n = M.n;
  const long long p = idx >> 6;
  const int j = (int)(idx & 63);
  if (p >= n) return;
  const long long e = p * MLP_WIDTH + j, ch = n * MLP_WIDTH;
  float g[JET];
  if constexpr (OUT) {
    const float* W = M.params + M.off_w[M.depth];
#pragma unroll
    for (int c = 0; c < JET; ++c) {
      float s = 0.0f;
#pragma unroll
      for (int o = 0; o < MLP_OUT; ++o) s = fmaf(G[(c * n + p) * MLP_OUT + o], W[j * MLP_OUT + o], s);
      g[c] = s;
    }
  } else {
#pragma unroll
    for (int c = 0; c < JET; ++c) g[c] = G[c * ch + e];
  }
  const float y = aj[e], tp = 1.0f - y * y;
  float d0 = g[0] * tp;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float zd = zj[d * ch + e], zdd = zj[(3 + d) * ch + e];
    const float gd = g[1 + d], gdd = g[4 + d];
    dz[(4 + d) * ch + e] = gdd * tp;
    dz[(1 + d) * ch + e] = gd * tp - 4.0f * gdd * y * tp * zd;
    d0 += -2.0f * y * tp * (gd * zd + gdd * zdd) - 2.0f * tp * (1.0f - 3.0f * y * y) * gdd * zd * zd;
  }
  dz[e] = d0;
}

// Boundary-type loss: per point sum_k ((out_k - target_k) / norm_k)^2 and its seed
// dL/dout_k = 2 (out_k - target_k) / norm_k^2; per-block partial sums of the loss.
__global__ __launch_bounds__(256) void k_mlp_fit_seed(long long n, const float* __restrict__ out,
                                                      const float* __restrict__ target, FitNorms inv,
                                                      float* __restrict__ dL, float* __restrict__ partials) {
  __shared__ float red[4];
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  float l = 0.0f;
  if (p < n) {
#pragma unroll
    for (int k = 0; k < MLP_OUT; ++k) {
      const float r = (out[p * MLP_OUT + k] - target[p * MLP_OUT + k]) * inv.v[k];
      l = fmaf(r, r, l);
      dL[p * MLP_OUT + k] = 2.0f * r * inv.v[k];
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0 && partials) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// fixed-order sum of the block partials into one value
__global__ __launch_bounds__(256) void k_sum_partials(const float* __restrict__ partials, int nblk,
                                                      float* __restrict__ result) {
  __shared__ float red[4];
  float s = 0.0f;
  for (int i = threadIdx.x; i < nblk; i += 256) s += partials[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *result = (red[0] + red[1]) + (red[2] + red[3]);
}

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int blocks_for(long long threads) { return (int)((threads + 255) / 256); }

// blocks (four wavefronts each) of the parameter-gradient reduction over `rows` rows: one
// per 64 rows, up to two per compute unit
inline long long wgrad_blocks(long long rows) {
  const long long b = (rows + 63) / 64;
  return b < 1 ? 1 : (b > 512 ? 512 : b);
}

}  // namespace

size_t mlp_work_bytes(int depth, long long n) {
  const long long nblk = wgrad_blocks(n);
  size_t b = 0;
  b += al256(sizeof(float) * (size_t)depth * (size_t)n * MLP_WIDTH);
  b += 2 * al256(sizeof(float) * (size_t)n * MLP_WIDTH);
  b += al256(sizeof(float) * (size_t)depth * MLP_WIDTH * MLP_WIDTH);
  b += al256(sizeof(float) * (size_t)(depth + 1) * (size_t)nblk * MLP_PART);
  b += al256(sizeof(float) * 4 * (size_t)n);
  return b;
}

void mlp_work_carve(void* ws, int depth, long long n, MlpWork& w) {
  const long long nblk = wgrad_blocks(n);
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
  p += al256(sizeof(float) * (size_t)depth * MLP_WIDTH * MLP_WIDTH);
  w.partial = reinterpret_cast<float*>(p);
  p += al256(sizeof(float) * (size_t)(depth + 1) * (size_t)nblk * MLP_PART);
  w.xh = reinterpret_cast<float*>(p);
}

hipError_t launch_mlp_forward(const MlpDev& M, const MlpWork& w, float* out, float* T, float T0, float dT,
                              hipStream_t stream) {
  if (M.n == 0) return hipSuccess;
  const size_t lds = sizeof(float) * (size_t)fused_lds_floats(M.depth);
  // up to 133 KB of staged weights (8 hidden layers): allow the kernel the largest size
  // once per device (safe from any thread)
  static std::atomic<int> lds_set[64];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64 || !lds_set[dev].load(std::memory_order_acquire)) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_forward_fused),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(float) * (size_t)fused_lds_floats(MLP_MAX_DEPTH)));
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) lds_set[dev].store(1, std::memory_order_release);
  }
  const long long groups = (M.n + 31) / 32;
  const long long blocks = (groups + 3) / 4;
  const int grid = (int)(blocks < 2048 ? blocks : 2048);
  hipLaunchKernelGGL(k_mlp_forward_fused, dim3(grid), dim3(256), lds, stream, M, w.act, w.xh, out, T, T0, dT);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const MlpDev& M, const MlpWork& w, const float* dL_dout, float* dparams,
                               hipStream_t stream) {
  if (M.n == 0) return hipSuccess;
  const long long n = M.n;
  const int D = M.depth;
  auto act = [&](int l) { return w.act + (size_t)(l - 1) * n * MLP_WIDTH; };  // a_l, l = 1 .. D
  auto part = [&](int l) { return w.partial + (size_t)l * w.nblk * MLP_PART; };
  hipLaunchKernelGGL(k_mlp_transpose, dim3(blocks_for((long long)D * MLP_WIDTH * MLP_WIDTH)), dim3(256), 0, stream, M,
                     w.wt);
  // output layer: dW_D = a_D^T dL, db_D = sum dL; delta_D = (dL W_D^T)(1 - a_D^2)
  hipLaunchKernelGGL((k_mlp_wgrad<false, PROD_DTANH>), dim3(w.nblk), dim3(256), 0, stream, M, act(D), dL_dout, MLP_OUT,
                     MLP_OUT, part(D), w.rows_per_block, n, n, w.wt + (size_t)(D - 1) * MLP_WIDTH * MLP_WIDTH,
                     w.delta[0]);
  int cur = 0;
  for (int l = D - 1; l >= 1; --l) {
    // dW_l = a_l^T delta_{l+1}; delta_l = (delta_{l+1} W_l^T)(1 - a_l^2)
    hipLaunchKernelGGL((k_mlp_wgrad<false, PROD_DTANH>), dim3(w.nblk), dim3(256), 0, stream, M, act(l), w.delta[cur],
                       MLP_WIDTH, MLP_WIDTH, part(l), w.rows_per_block, n, n,
                       w.wt + (size_t)(l - 1) * MLP_WIDTH * MLP_WIDTH, w.delta[cur ^ 1]);
    cur ^= 1;
  }
  hipLaunchKernelGGL((k_mlp_wgrad<true>), dim3(w.nblk), dim3(256), 0, stream, M, w.xh, w.delta[cur], MLP_WIDTH,
                     MLP_WIDTH, part(0), w.rows_per_block, n, n);
  for (int l = 0; l <= D; ++l) {
    const int fi = l == 0 ? 3 : MLP_WIDTH, fo = l == D ? MLP_OUT : MLP_WIDTH;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((fi * fo + fo + 15) / 16), dim3(256), 0, stream, part(l), w.nblk, fi, fo,
                       dparams + M.off_w[l], dparams + M.off_b[l]);
  }
  return hipGetLastError();
}

size_t mlp_jet_work_bytes(int depth, long long n) {
  const long long rows = JET * n;
  const long long nblk = wgrad_blocks(rows);
  size_t b = 0;
  b += al256(sizeof(float) * (size_t)depth * JET * (size_t)n * MLP_WIDTH);        // a jets
  b += al256(sizeof(float) * (size_t)depth * (JET - 1) * (size_t)n * MLP_WIDTH);  // z jets
  b += 2 * al256(sizeof(float) * JET * (size_t)n * MLP_OUT);                      // output jets, seeds
  b += 3 * al256(sizeof(float) * JET * (size_t)n * MLP_WIDTH);                    // dz x 2, G
  b += al256(sizeof(float) * (size_t)depth * MLP_WIDTH * MLP_WIDTH);
  b += al256(sizeof(float) * (size_t)(depth + 1) * (size_t)nblk * MLP_PART);
  b += al256(sizeof(float) * (size_t)((n + 255) / 256 + 1));
  b += al256(sizeof(float) * 4 * (size_t)n);
  return b;
}

hipError_t launch_mlp_pde(const MlpDev& M, void* ws, const PdeConst& P, float* loss, float* dparams, float* residuals,
                          hipStream_t stream) {
  const long long n = M.n;
  const int D = M.depth;
  if (n == 0) {
    if (loss) hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, stream, (const float*)nullptr, 0, loss);
    return hipGetLastError();
  }
  const long long rows = JET * n;
  const long long nblk = wgrad_blocks(rows);
  const long long rpb = ((rows + nblk - 1) / nblk + 63) / 64 * 64;
  unsigned char* q = static_cast<unsigned char*>(ws);
  auto take = [&](size_t bytes) {
    float* f = reinterpret_cast<float*>(q);
    q += al256(bytes);
    return f;
  };
  const size_t chw = sizeof(float) * (size_t)n * MLP_WIDTH;
  float* aj = take(chw * JET * D);
  float* zj = take(chw * (JET - 1) * D);
  float* oj = take(sizeof(float) * JET * (size_t)n * MLP_OUT);
  float* dj = take(sizeof(float) * JET * (size_t)n * MLP_OUT);
  float* dz[2] = {take(chw * JET), take(chw * JET)};
  float* G = take(chw * JET);
  float* wt = take(sizeof(float) * (size_t)D * MLP_WIDTH * MLP_WIDTH);
  float* partial = take(sizeof(float) * (size_t)(D + 1) * (size_t)nblk * MLP_PART);
  float* lpart = take(sizeof(float) * (size_t)((n + 255) / 256 + 1));
  float* xh = take(sizeof(float) * 4 * (size_t)n);
  auto A = [&](int l) { return aj + (size_t)(l - 1) * JET * n * MLP_WIDTH; };       // a_l jets, l = 1 .. D
  auto Z = [&](int l) { return zj + (size_t)(l - 1) * (JET - 1) * n * MLP_WIDTH; };  // z_l jets
  auto part = [&](int l) { return partial + (size_t)l * nblk * MLP_PART; };
  const unsigned tiles = (unsigned)((n + 127) / 128);
  // forward
  hipLaunchKernelGGL(k_jet_first, dim3(blocks_for(n * MLP_WIDTH)), dim3(256), 0, stream, M, A(1), Z(1), xh);
  for (int l = 1; l < D; ++l)
    hipLaunchKernelGGL(k_jet_dense, dim3(tiles, 3), dim3(256), 0, stream, n, A(l), M.params + M.off_w[l],
                       M.params + M.off_b[l], A(l + 1), Z(l + 1));
  hipLaunchKernelGGL(k_jet_out, dim3(blocks_for(rows * 8)), dim3(256), 0, stream, M, A(D), oj);
  hipLaunchKernelGGL(k_pde_seed, dim3(blocks_for(n)), dim3(256), 0, stream, n, oj, P, dparams ? dj : nullptr,
                     residuals, lpart);
  if (loss) hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, stream, lpart, blocks_for(n), loss);
  if (!dparams) return hipGetLastError();
  // reverse
  hipLaunchKernelGGL(k_mlp_transpose, dim3(blocks_for((long long)D * MLP_WIDTH * MLP_WIDTH)), dim3(256), 0, stream, M,
                     wt);
  hipLaunchKernelGGL((k_mlp_wgrad<false>), dim3((unsigned)nblk), dim3(256), 0, stream, M, A(D), dj, MLP_OUT, MLP_OUT,
                     part(D), rpb, rows, n);
  hipLaunchKernelGGL((k_jet_act_back<true>), dim3(blocks_for(n * MLP_WIDTH)), dim3(256), 0, stream, M, dj, A(D),
                     Z(D), dz[0]);
  int cur = 0;
  for (int l = D - 1; l >= 1; --l) {
    // dW_l = sum_c a_l^c^T dz_{l+1}^c (bias: value channel); G = dz_{l+1} W_l^T; dz_l
    hipLaunchKernelGGL((k_mlp_wgrad<false, PROD_PLAIN>), dim3((unsigned)nblk), dim3(256), 0, stream, M, A(l), dz[cur],
                       MLP_WIDTH, MLP_WIDTH, part(l), rpb, rows, n, wt + (size_t)(l - 1) * MLP_WIDTH * MLP_WIDTH, G);
    hipLaunchKernelGGL((k_jet_act_back<false>), dim3(blocks_for(n * MLP_WIDTH)), dim3(256), 0, stream, M, G, A(l),
                       Z(l), dz[cur ^ 1]);
    cur ^= 1;
  }
  // first layer: the input jet (xhat, e_d, 0): rows 0 .. 4n of dz_1
  hipLaunchKernelGGL((k_mlp_wgrad<true>), dim3((unsigned)nblk), dim3(256), 0, stream, M, xh, dz[cur], MLP_WIDTH,
                     MLP_WIDTH, part(0), rpb, 4 * n, n);
  for (int l = 0; l <= D; ++l) {
    const int fi = l == 0 ? 3 : MLP_WIDTH, fo = l == D ? MLP_OUT : MLP_WIDTH;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((fi * fo + fo + 15) / 16), dim3(256), 0, stream, part(l), (int)nblk, fi,
                       fo, dparams + M.off_w[l], dparams + M.off_b[l]);
  }
  return hipGetLastError();
}

hipError_t launch_mlp_fit_seed(long long n, const float* out, const float* target, const double* norms, float* dL_dout,
                               float* loss, float* partials, hipStream_t stream) {
  FitNorms inv;
  for (int k = 0; k < MLP_OUT; ++k) inv.v[k] = (float)(1.0 / norms[k]);
  const int nblk = blocks_for(n);
  if (n > 0)
    hipLaunchKernelGGL(k_mlp_fit_seed, dim3(nblk), dim3(256), 0, stream, n, out, target, inv, dL_dout,
                       loss ? partials : nullptr);
  if (loss) hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, stream, partials, n > 0 ? nblk : 0, loss);
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
