/*
 * bos_oracle.h -- FP64 CPU oracle for single-view BOS ray tracing.
 *
 * TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load this library. It shares no code, header or constant with the
 * GPU library; the two see the same input arrays and nothing else.
 *
 * Conventions: metres, world frame, z up. Fields are eta - 1 ("delta") at voxel
 * centres, indexed [nz][ny][nx] (x fastest); voxel i on an axis of n voxels over
 * [lo, hi] sits at lo + (i + 1/2)(hi - lo)/n. Pixel j = row * width + col, row 0 at
 * the top. All functions return 0 on success and a negative value on bad arguments.
 */
#ifndef BOS_ORACLE_H
#define BOS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_FIELD_GRID = 0, OR_FIELD_HOMOGENEOUS = 1, OR_FIELD_LINEAR = 2,
       OR_FIELD_ETA2_LINEAR = 3, OR_FIELD_GAUSSIAN = 4 };

enum { OR_RAY_MISSED_BOX = 1, OR_RAY_TRUNCATED = 2, OR_RAY_NO_WALL_HIT = 4,
       OR_RAY_NONFINITE = 8, OR_RAY_OFF_PATTERN = 16 };

enum { OR_WALL_PRINTED = 0, OR_WALL_PROJECTOR = 1 };

enum { OR_CODE_F32 = 0, OR_CODE_F16 = 1, OR_CODE_BF16 = 2 };

/* Ray integration, Sec. 2.B: nonlinear (Eq. 1 fully coupled, the force sampled at the
   state) or quasi-linear (the force sampled on the straight line from the entry state). */
enum { OR_TRACER_NONLINEAR = 0, OR_TRACER_QUASILINEAR = 1 };

typedef struct {
  int32_t mode;          /* OR_FIELD_* */
  int32_t n[3];          /* voxels per axis (grid mode), each >= 2 */
  double lo[3], hi[3];   /* the field box */
  const double* delta;   /* grid mode: eta - 1 at voxel centres [nz][ny][nx] */
  /* analytic parameters:
       HOMOGENEOUS  delta = a
       LINEAR       delta = a + g.(x - c)
       ETA2_LINEAR  eta^2 = a + g.(x - c), delta = eta - 1
       GAUSSIAN     delta = a + eps * exp(-|x - c|^2 / (2 sigma^2)) */
  double a, g[3], c[3], sigma, eps;
  /* one-voxel perturbation used by finite differences: delta[pert_index] += pert_value */
  int64_t pert_index;
  double pert_value;
} or_field;

typedef struct {
  int32_t width, height;
  double cam_pos[3], cam_fwd[3], cam_right[3], cam_up[3], fov_x_deg;
  double wall_origin[3], wall_normal[3], wall_u[3], wall_v[3];
  int32_t wall_mode, pat_w, pat_h;
  double pat_extent_u, pat_extent_v;
  double proj_pos[3], proj_fwd[3], proj_right[3], proj_up[3], proj_fov_x_deg;
  double step;           /* RK4 step h in the ray parameter t */
  int32_t max_steps;
  int32_t tracer;        /* OR_TRACER_* */
  /* Eq. (2) pixel integral: spp rays per pixel (1: one ray through the pixel centre),
     sub-pixel offsets from Philox-4x32-10 keyed by seed with the triangular filter;
     radiometry != 0 weights each ray by |<n_w, v_w>| / (length of the ray path). Rays
     are sample-major: ray r = s * P + i is sample s of pixel i (pixel_ids[i] or i). */
  int32_t spp;
  uint32_t seed;
  int32_t radiometry;
  const double* pattern; /* [pat_h][pat_w], row 0 at the top */
} or_scene;

int or_version(void);
int or_threads(void);

/* Sec. 2.A: eta - 1 = rho0 G T0 / T, in binary64 (exact reference) ... */
int or_delta_from_temperature(const float* T, int64_t n, double rho0G, double T0, double* delta);
/* ... and in binary32 as two correctly rounded operations, rho0G * (T0 / T), which is
   the arithmetic that decides stored codes. */
int or_delta_from_temperature_f32(const float* T, int64_t n, float rho0G, float T0, float* delta);
/* Storage codes q = RN_even(s (delta - c)) (binary32 subtract and scale, then one rounding
   to the code type); codes are float32 or uint16 bit patterns. */
int or_encode(const float* delta, int64_t n, int32_t code, double scale, double offset, void* codes);
/* delta = c + q / s, exact in binary64. */
int or_decode(const void* codes, int64_t n, int32_t code, double scale, double offset, double* delta);

/* Field sampler: delta, gradient and Hessian (row-major 3x3) at P. */
int or_sample(const or_field* F, const double* P, double* delta, double* grad, double* hess);
/* Pinhole camera ray through a pixel centre. */
int or_camera_ray(const or_scene* S, int32_t pixel, double* org, double* dir);
/* nsteps Sharma steps from (x0, v0) with no box and no exit test. */
int or_integrate(const or_field* F, const double* x0, const double* v0, double h, int32_t nsteps,
                 double* x_out, double* v_out);
/* nsteps quasi-linear steps from (x0, v0): forces on the line x0 + v0 t. */
int or_integrate_quasi(const or_field* F, const double* x0, const double* v0, double h, int32_t nsteps,
                       double* x_out, double* v_out);

/* Forward: per ray wall coordinates (u, v), deflection (u, v) - (u0, v0) against the
   undeflected camera ray, step count and status. exit_xv (nullable) gets [x(3), v(3)]
   at the last integrated state, vdir (nullable) the unit direction at the wall, path
   (nullable) the length of the ray path: the polyline from the camera centre through
   the box entry and every integrated state, plus the signed straight continuation
   s |v| to the wall hit (s < 0 when the last step ended past the wall plane). pixel_ids NULL means all
   width*height pixels. */
int or_trace(const or_field* F, const or_scene* S, const int32_t* pixel_ids, int32_t n_rays,
             double* uv, double* duv, int32_t* n_steps, uint8_t* status, double* exit_xv, double* vdir,
             double* path);
/* Wall luminance at each ray's hit and its derivative w.r.t. (u, v). status is updated
   with OR_RAY_OFF_PATTERN. */
int or_render(const or_scene* S, const int32_t* pixel_ids, int32_t n_rays, const double* uv,
              uint8_t* status, double* image, double* dI_duv);
/* L_BOS = sum_j (image_j - target_j)^2 and dL/d(u, v) = 2 r_j dI/d(u, v). */
int or_loss(const double* image, const double* target, const double* dI_duv, int32_t n,
            double* loss, double* dL_duv);
/* Eq. (2) per pixel: image_i = (1/spp) sum_s I_r over the pixel's rays r = s P + i, with
   I_r = L_wall(u, v) (times |<n_w, vdir>| / path with radiometry); per ray
   dI_duv = (1/spp) dI_r/d(u, v) and, with radiometry, dI_ddir = (1/spp) dI_r/d(vdir) and
   dI_dpath = (1/spp) dI_r/d(path), vdir and path from or_trace (both may be NULL
   without radiometry). */
int or_render_pixels(const or_scene* S, int32_t n_pixels, const double* uv, const double* vdir, const double* path,
                     uint8_t* status, double* image, double* dI_duv, double* dI_ddir, double* dI_dpath);
/* L_BOS over pixels and per ray dL/d(u, v) = 2 r_i dI_duv (dL/d vdir, dL/d path likewise;
   each output nullable). */
int or_loss_pixels(const double* image, const double* target, int32_t n_pixels, int32_t spp, const double* dI_duv,
                   const double* dI_ddir, const double* dI_dpath, double* loss, double* dL_duv, double* dL_ddir,
                   double* dL_dpath);
/* Exact gradient of sum_r dL_duv_r . (u_r, v_r) + dL_ddir_r . vdir_r + dL_dpath_r path_r
   (dL_ddir, dL_dpath may be NULL) w.r.t. every voxel, ADDED into grad. */
int or_adjoint(const or_field* F, const or_scene* S, const int32_t* pixel_ids, int32_t n_rays,
               const double* dL_duv, const double* dL_ddir, const double* dL_dpath, double* grad);
/* Tangent-linear model: d(u, v)/d(delta) (and d vdir/d(delta), d path/d(delta), both
   nullable) applied to the voxel perturbation vfield. */
int or_tangent(const or_field* F, const or_scene* S, const int32_t* pixel_ids, int32_t n_rays,
               const double* vfield, double* duv_dot, double* ddir_dot, double* dpath_dot);
/* Philox-4x32-10 (Salmon et al., SC'11) of a 128-bit counter under a 64-bit key. */
int or_philox4x32(const uint32_t* ctr, const uint32_t* key, uint32_t* out);
/* Sub-pixel offset (pixels, in [-1, 1]^2) of sample s of pixel p: two 24-bit uniforms from
   Philox(counter (p, s, 0, 0), key (seed, 0)), each mapped through the inverse CDF of
   the triangular filter. */
int or_sample_offset(uint32_t seed, int32_t pixel, int32_t sample, double* ox, double* oy);
/* Central finite differences of L_BOS w.r.t. single voxels. locked != 0 freezes every
   branch of the unperturbed run (interpolation cells, clamp flags, step counts, texel
   cells) so that the difference quotient sees only the smooth dependence. */
int or_fd_voxels(const or_field* F, const or_scene* S, const int32_t* pixel_ids, int32_t n_rays,
                 const double* target, const int64_t* voxels, int32_t n_vox, double h,
                 int32_t locked, double* fd);

#ifdef __cplusplus
}
#endif
#endif
