// mlp_launch.hpp -- host-side descriptor and launches of the network-field kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace rbos {

constexpr int MLP_WIDTH = 64;     // hidden units per layer
constexpr int MLP_OUT = 5;        // T_nd, p, u_x, u_y, u_z
constexpr int MLP_MAX_DEPTH = 8;  // hidden layers

// One evaluation set of the MLP: its parameters and where its points come from.
struct MlpDev {
  int depth;                      // hidden layers (>= 1)
  const float* params;            // packed: per layer W [in][out] row-major, then b [out]
  int off_w[MLP_MAX_DEPTH + 1];   // float offsets of each layer's W and b
  int off_b[MLP_MAX_DEPTH + 1];
  long long n;                    // points
  const float* points;            // [n][3] metres, or nullptr: the voxel centres of the grid below
  int nx, ny, nz;                 // grid mode: voxel counts (points in x-fastest order)
  float xs[3], xo[3];             // points mode: xhat = x * xs + xo
};

// Workspace carve-up for one point set (all float arrays, 256-byte aligned):
// activations a_1 .. a_depth [n][64], two delta buffers [n][64], transposed hidden
// weights (depth - 1) x [64][64], per-block partial parameter gradients and the
// normalised inputs [n][4].
struct MlpWork {
  float* act;       // depth x [n][64]
  float* delta[2];  // [n][64]
  float* wt;        // (depth - 1) x [64][64]
  float* partial;   // (depth + 1) x nblk x MLP_PART floats
  float* xh;        // [n][4] normalised inputs (fourth column 0)
  int nblk;         // blocks of the parameter-gradient reduction
  long long rows_per_block;
};
constexpr int MLP_PART = 64 * 64 + 64;  // one layer's partial dW (up to 64 x 64) and db

size_t mlp_work_bytes(int depth, long long n);
void mlp_work_carve(void* ws, int depth, long long n, MlpWork& w);

// forward: activations into the workspace; out [n][5] and T = T0 + dT * out0 (both
// nullable)
hipError_t launch_mlp_forward(const MlpDev& M, const MlpWork& w, float* out, float* T, float T0, float dT,
                              hipStream_t stream);
// backward from dL/dout [n][5] (activations of the matching forward in the workspace):
// dparams += the parameter gradient
hipError_t launch_mlp_backward(const MlpDev& M, const MlpWork& w, const float* dL_dout, float* dparams,
                               hipStream_t stream);
// dL/dout at the voxel centres from dL/d(eta - 1): channel 0 = grad * (-rho0G T0 / T^2) * dT,
// the other channels 0
hipError_t launch_mlp_bos_seed(long long n, const float* T, const double* grad_delta, double rho0G, double T0,
                               double dT, float* dL_dout, hipStream_t stream);

// boundary-type loss sum_points sum_k ((out_k - target_k) / norm_k)^2: seed dL/dout and
// (nullable) the loss, reduced in a fixed order through `partials` (one float per 256
// points)
struct FitNorms {
  float v[MLP_OUT];  // 1 / norm_k
};
hipError_t launch_mlp_fit_seed(long long n, const float* out, const float* target, const double* norms, float* dL_dout,
                               float* loss, float* partials, hipStream_t stream);

// PDE loss (Sec. 2.D) on the jets of the MLP: s_d = d xhat_d / d x_nd = 2 L / (hi - lo)
struct PdeConst {
  float s[3];
  float inv_re, inv_pe, ri;
  float g[3];  // weights of the mass, momentum and heat residuals
};
size_t mlp_jet_work_bytes(int depth, long long n);
// forward jets, residuals [n][5] (nullable), loss (nullable) and, with dparams, the
// parameter gradient added into dparams
hipError_t launch_mlp_pde(const MlpDev& M, void* ws, const PdeConst& P, float* loss, float* dparams, float* residuals,
                          hipStream_t stream);

}  // namespace rbos
