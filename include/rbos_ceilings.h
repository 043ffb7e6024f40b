/*
 * rbos_ceilings.h -- C ABI of librbos_ceilings.so: microbenchmarks that measure the
 * ceilings the ray-tracing kernels of librbos are compared with on the GPU at hand.
 * They are measurement tools, not part of the method. Every pointer is device memory
 * owned by the caller; each call enqueues one kernel on `stream` (a hipStream_t) and
 * returns 0, -2 for invalid arguments (nothing enqueued) or -6 if the launch failed.
 */
#ifndef RBOS_CEILINGS_H
#define RBOS_CEILINGS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Coherent cell-record gathers in the tracers' access pattern: 8 x 8 ray tiles of a
   width x height image spread over the x-z face of a px * py * pz record grid
   (rec_bytes = 32 or 16 per record, x fastest); each ray walks along +y in half-record
   steps and reads the records of three points per step. Delivered bytes =
   width * height * steps * 3 * rec_bytes. out: [ceil(width/8) * ceil(height/8) * 64]
   floats. px, py, pz >= 4. */
int ceil_gather_coherent(const void* records, int rec_bytes, int px, int py, int pz, int width, int height,
                         int steps, float* out, void* stream);

/* Scattered gathers: blocks * 256 lanes each read `iters` pseudo-random records among the
   first 2^log2_n_rec (1 .. 27; iters a multiple of 4). Delivered bytes =
   blocks * 256 * iters * rec_bytes. out: [blocks * 256] floats. */
int ceil_gather_scattered(const void* records, int rec_bytes, int log2_n_rec, int blocks, int iters, float* out,
                          void* stream);

/* Plain FP32 fused multiply-adds: blocks * 256 lanes x iters x 16 chains.
   Flops = blocks * 256 * iters * 32. out: [blocks * 256] floats. */
int ceil_fma(float* out, int blocks, int iters, void* stream);

/* FP64 atomic adds into grad [nz][ny][nx] (each 8 lanes add 1.0 to the 8 corner voxels of
   one pseudo-random cell): blocks * 256 * iters atomics. grad must be coarse-grained
   device memory. */
int ceil_atomic_f64(double* grad, int nx, int ny, int nz, int blocks, int iters, void* stream);

/* Stream copy of `bytes` (a multiple of 16) from src to dst with a grid-stride loop. */
int ceil_copy(const void* src, void* dst, size_t bytes, int blocks, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RBOS_CEILINGS_H */
