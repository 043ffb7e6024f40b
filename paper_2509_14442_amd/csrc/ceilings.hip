// ceilings.hip -- microbenchmarks that measure, on the GPU at hand, the ceilings the
// tracer kernels are compared with: the delivered bandwidth of coherent and of scattered
// 32-byte (16-byte) cell-record gathers, the FP32 fused multiply-add rate of plain
// (unpacked) VALU code, device-scope FP64 atomic adds into a voxel gradient, and an HBM
// stream copy. Not part of the method: bench.py times these next to the tracer kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rbos_ceilings.h"

namespace {

#define CEIL_GLOBAL __attribute__((address_space(1)))
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 ld4(const f32x4* p) { return *(const CEIL_GLOBAL f32x4*)p; }

// 32-bit linear congruential step (Numerical Recipes constants) for scattered addresses
__device__ __forceinline__ unsigned lcg(unsigned x) { return x * 1664525u + 1013904223u; }

// Coherent gathers in the tracers' pattern: a wavefront is an 8 x 8 tile of rays of a
// width x height image spread over the x-z face of a record grid (px, py, pz records per
// axis), each ray runs along +y in steps of half a record and gathers the records of
// three points per step, a quarter record apart (the three samples of one Sharma step).
// Record indices are clamped into the grid. rec_bytes is 32 (two 16-byte loads) or 16.
template <int REC_BYTES>
__global__ __launch_bounds__(256) void k_gather_coherent(const unsigned char* __restrict__ rec, int px, int py,
                                                         int pz, int width, int height, int steps,
                                                         float* __restrict__ out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + wave;
  const int tiles_x = (width + 7) / 8;
  const int col = (tile % tiles_x) * 8 + (lane & 7), row = (tile / tiles_x) * 8 + (lane >> 3);
  if (row >= height) return;
  const float x = 1.0f + (col + 0.5f) * (float)(px - 3) / (float)width;
  const float z = 1.0f + (row + 0.5f) * (float)(pz - 3) / (float)height;
  const unsigned ix = (unsigned)min(max((int)x, 0), px - 1);
  const unsigned iz = (unsigned)min(max((int)z, 0), pz - 1);
  const unsigned base = ix + (unsigned)px * (unsigned)py * iz;
  const int ny_walk = 2 * (py - 3);  // half-record steps along y before wrapping
  float acc = 0.0f;
  int k = 0;
  for (int s = 0; s < steps; ++s) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const float y = 1.0f + 0.5f * (float)k + 0.25f * (float)q;
      const unsigned iy = (unsigned)min((int)y, py - 1);
      const unsigned r = base + iy * (unsigned)px;
      const f32x4* p = reinterpret_cast<const f32x4*>(rec + (size_t)r * REC_BYTES);
      const f32x4 a = ld4(p);
      acc += (a.x + a.y) + (a.z + a.w);
      if constexpr (REC_BYTES == 32) {
        const f32x4 b = ld4(p + 1);
        acc += (b.x + b.y) + (b.z + b.w);
      }
    }
    k = k + 1 == ny_walk ? 0 : k + 1;
  }
  out[(size_t)tile * 64 + lane] = acc;
}

// Scattered gathers: every lane reads pseudo-random records among the first 2^log2_n
// records, so nearly every access is a separate cache line (a footprint that fits the L2
// measures its request rate, a larger one the MALL / HBM).
template <int REC_BYTES>
__global__ __launch_bounds__(256) void k_gather_scattered(const unsigned char* __restrict__ rec, int log2_n,
                                                          int iters, float* __restrict__ out) {
  const unsigned tid = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned x = lcg(tid * 2654435761u);
  float acc = 0.0f;
  for (int it = 0; it < iters; it += 4) {
    unsigned r[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x = lcg(x);
      r[u] = x >> (32 - log2_n);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const f32x4* p = reinterpret_cast<const f32x4*>(rec + (size_t)r[u] * REC_BYTES);
      const f32x4 a = ld4(p);
      acc += (a.x + a.y) + (a.z + a.w);
      if constexpr (REC_BYTES == 32) {
        const f32x4 b = ld4(p + 1);
        acc += (b.x + b.y) + (b.z + b.w);
      }
    }
  }
  out[tid] = acc;
}

// 16 independent chains of plain FP32 FMAs per lane (compiled without packed FP32
// instructions, so each is one v_fma_f32).
__global__ __launch_bounds__(256) void k_fma(float* __restrict__ out, int iters, float a, float b) {
  float x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = (float)(threadIdx.x + i) * 1e-3f;
#pragma unroll 4
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = fmaf(x[i], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) s += x[i];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// FP64 atomic adds into an nx*ny*nz gradient in the adjoint's pattern: each group of 8
// lanes adds to the 8 corner voxels of one pseudo-random cell.
__global__ __launch_bounds__(256) void k_atomic_f64(double* __restrict__ g, int nx, int ny, int nz, int iters) {
  const unsigned tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int corner = threadIdx.x & 7;
  const unsigned cells = (unsigned)(nx - 1) * (unsigned)(ny - 1) * (unsigned)(nz - 1);
  unsigned x = lcg((tid >> 3) * 2654435761u);
  for (int it = 0; it < iters; ++it) {
    x = lcg(x);
    const unsigned c = x % cells;
    const unsigned cx = c % (unsigned)(nx - 1), t = c / (unsigned)(nx - 1);
    const unsigned cy = t % (unsigned)(ny - 1), cz = t / (unsigned)(ny - 1);
    const size_t v = ((size_t)(cz + (corner >> 2)) * ny + (cy + ((corner >> 1) & 1))) * nx + cx + (corner & 1);
    __builtin_amdgcn_global_atomic_fadd_f64((CEIL_GLOBAL double*)(g + v), 1.0);
  }
}

// Stream copy: each lane moves 4 x 16 bytes per round (four loads in flight before the
// stores), rounds striding over the grid.
__global__ __launch_bounds__(256) void k_copy(const f32x4* __restrict__ src, f32x4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const f32x4 a = ld4(src + i), b = ld4(src + i + stride), c = ld4(src + i + 2 * stride),
                d = ld4(src + i + 3 * stride);
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = ld4(src + i);
}

int status(hipError_t e) { return e == hipSuccess ? 0 : -6; }

}  // namespace

extern "C" {

int ceil_gather_coherent(const void* records, int rec_bytes, int px, int py, int pz, int width, int height,
                         int steps, float* out, void* stream) {
  if (!records || !out || (rec_bytes != 32 && rec_bytes != 16) || px < 4 || py < 4 || pz < 4 || width < 1 ||
      height < 1 || steps < 1)
    return -2;
  const int tiles = ((width + 7) / 8) * ((height + 7) / 8);
  const dim3 grid((tiles + 3) / 4), block(256);
  const unsigned char* r = static_cast<const unsigned char*>(records);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (rec_bytes == 32)
    hipLaunchKernelGGL(k_gather_coherent<32>, grid, block, 0, s, r, px, py, pz, width, height, steps, out);
  else
    hipLaunchKernelGGL(k_gather_coherent<16>, grid, block, 0, s, r, px, py, pz, width, height, steps, out);
  return status(hipGetLastError());
}

int ceil_gather_scattered(const void* records, int rec_bytes, int log2_n_rec, int blocks, int iters, float* out,
                          void* stream) {
  if (!records || !out || (rec_bytes != 32 && rec_bytes != 16) || log2_n_rec < 1 || log2_n_rec > 27 ||
      blocks < 1 || iters < 4 || iters % 4 != 0)
    return -2;
  const unsigned char* r = static_cast<const unsigned char*>(records);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (rec_bytes == 32)
    hipLaunchKernelGGL(k_gather_scattered<32>, dim3(blocks), dim3(256), 0, s, r, log2_n_rec, iters, out);
  else
    hipLaunchKernelGGL(k_gather_scattered<16>, dim3(blocks), dim3(256), 0, s, r, log2_n_rec, iters, out);
  return status(hipGetLastError());
}

int ceil_fma(float* out, int blocks, int iters, void* stream) {
  if (!out || blocks < 1 || iters < 1) return -2;
  hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), out, iters, 0.999f,
                     1e-3f);
  return status(hipGetLastError());
}

int ceil_atomic_f64(double* grad, int nx, int ny, int nz, int blocks, int iters, void* stream) {
  if (!grad || nx < 2 || ny < 2 || nz < 2 || blocks < 1 || iters < 1) return -2;
  hipLaunchKernelGGL(k_atomic_f64, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), grad, nx, ny, nz,
                     iters);
  return status(hipGetLastError());
}

int ceil_copy(const void* src, void* dst, size_t bytes, int blocks, void* stream) {
  if (!src || !dst || bytes % 16 != 0 || blocks < 1) return -2;
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const f32x4*>(src), static_cast<f32x4*>(dst), bytes / 16);
  return status(hipGetLastError());
}

}  // extern "C"
