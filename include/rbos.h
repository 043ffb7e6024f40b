/*
 * rbos.h -- C ABI of the MI355X (gfx950) BOS ray-tracing library librbos.so.
 *
 * What it computes (Teh, Ali, Rapp, Mansour, "Indoor Airflow Imaging Using
 * Physics-Informed Background-Oriented Schlieren Tomography"):
 *   - Sec. 2.A: the refractive index of air from temperature, eta = 1 + rho0 G T0 / T,
 *     stored per voxel as eta - 1 (optionally scaled into FP16 / BF16 codes);
 *   - Sec. 2.B, Eq. (1): camera rays traced through the voxelised field with
 *     dx/dt = v, dv/dt = eta grad(eta) ("nonlinear ray tracing"), integrated with
 *     Sharma's three-stage Runge-Kutta-Nystrom scheme on the trilinear interpolant of
 *     the cell-centred grid (clamped to the edge values outside the voxel centres);
 *     rays start at the box entry with |v| = eta, move straight outside the box;
 *   - Sec. 2.C, Eq. (2): each pixel is the mean of spp rays cast through sub-pixel
 *     points drawn from the triangular camera filter (one ray through the centre when
 *     spp = 1); each ray carries the back wall's radiance at its hit, the printed
 *     texture or the pinhole projector's image (bilinear, zero outside), optionally
 *     weighted by |<n_w, v_w>| / ell (wall normal n_w, unit direction v_w at the wall,
 *     ell the length of the ray path, evaluated as the distance |X_w - c| from the
 *     camera centre c to the hit: the traced path is longer by a term of second order
 *     in the deflection angle, ~1e-11 relative for air);
 *   - Sec. 2.D: L_BOS = sum_j (I_flow^j - I^j(eta))^2, and its exact gradient with
 *     respect to eta - 1 at every voxel, back-propagated through the integrator from
 *     ray-state checkpoints (the gradient the paper obtains by automatic
 *     differentiation / the adjoint state method, here for the discrete scheme).
 *
 * Conventions
 *   - Units are metres in one world frame. Fields are indexed [nz][ny][nx] (x fastest);
 *     voxel i on an axis of n voxels over [lo, hi] has its centre at
 *     lo + (i + 1/2)(hi - lo)/n.
 *   - Pixel j = row * width + col, row 0 at the top of the image; the camera has a
 *     horizontal field of view and square pixels.
 *   - A scene traces n_pixels pixels (pixel_ids[i], or pixel i of the full image) with
 *     spp rays each: n_rays = n_pixels * spp rays, sample-major, ray r = s * n_pixels + i
 *     being sample s of pixel i. Per-ray arrays hold n_rays entries, per-pixel arrays
 *     (image, target) n_pixels.
 *   - Pointers marked [dev] are device memory owned by the caller. The library never
 *     allocates, frees or synchronises; every launch goes on the `stream` argument
 *     (a hipStream_t; NULL is the default stream), so all calls may be captured in a
 *     hipGraph.
 *   - Errors: argument validation happens on the host before anything is enqueued and
 *     returns a negative rbos_status; rbos_last_error() then describes it. A failed
 *     kernel launch returns RBOS_E_HIP. Faults inside kernels surface at the caller's
 *     next synchronisation. Per-ray conditions are reported in the status array, never
 *     through the return code.
 *   - Thread safety: calls on distinct streams with distinct workspaces may run
 *     concurrently. Outputs must not alias inputs.
 */
#ifndef RBOS_H
#define RBOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBOS_ABI_VERSION 2

typedef enum {
  RBOS_OK = 0,
  RBOS_E_NULL = -1,        /* a required pointer is NULL */
  RBOS_E_SHAPE = -2,       /* sizes inconsistent or outside the supported range */
  RBOS_E_RANGE = -3,       /* a value is out of range (non-finite, non-positive, ...) */
  RBOS_E_DTYPE = -4,       /* unknown storage type */
  RBOS_E_WORKSPACE = -5,   /* workspace NULL or smaller than rbos_workspace_bytes() */
  RBOS_E_HIP = -6,         /* a HIP runtime call failed */
  RBOS_E_UNSUPPORTED = -7  /* valid but unsupported option (e.g. checkpoint stride) */
} rbos_status;

/* storage format of the field: the type of the codes q (eta - 1 = enc_offset + q /
   enc_scale) and their layout. RBOS_F32 / F16 / BF16 store cell records (the 8 corner
   codes of every interpolation cell together: one load per sample, 8 copies of every
   voxel); the *_XPAIR formats store each voxel with its +x neighbour (four loads per
   sample, 2 copies of every voxel). See rbos_field_bytes. */
enum {
  RBOS_F32 = 0,
  RBOS_F16 = 1,
  RBOS_BF16 = 2,
  RBOS_F32_XPAIR = 3,
  RBOS_F16_XPAIR = 4,
  RBOS_BF16_XPAIR = 5
};

/* back-wall luminance model (Sec. 2.C) */
enum { RBOS_WALL_PRINTED = 0, RBOS_WALL_PROJECTOR = 1 };

/* ray integration (Sec. 2.B): NONLINEAR integrates Eq. (1) fully coupled, the force taken
   at the traced state; QUASILINEAR takes the force on the straight line x0 + v0 t from
   the entry state (x0, v0) at the same stage times, which drives velocity and position
   with the same Sharma update (two field samples per step, no state-dependent gathers). */
enum { RBOS_TRACER_NONLINEAR = 0, RBOS_TRACER_QUASILINEAR = 1 };

/* per-ray status bits */
enum {
  RBOS_RAY_MISSED_BOX = 1,  /* camera ray does not meet the field box: straight, 0 steps */
  RBOS_RAY_TRUNCATED = 2,   /* max_steps reached inside the box; continues straight */
  RBOS_RAY_NO_WALL_HIT = 4, /* final direction does not face the wall; rendered as 0 */
  RBOS_RAY_NONFINITE = 8,   /* state became NaN/Inf (non-finite field values) */
  RBOS_RAY_OFF_PATTERN = 16 /* wall point maps outside the pattern (set by rbos_render) */
};

/* Largest voxel count per axis. Positions are carried in grid units with an exact
   straight-line base that needs |coordinate| < 512. */
#define RBOS_MAX_DIM 448

/* One acquisition (host struct). Geometry in metres, world frame. */
typedef struct rbos_scene {
  /* field: nx*ny*nz voxels (each in [2, RBOS_MAX_DIM]) on the box [box_lo, box_hi] */
  int32_t nx, ny, nz;
  double box_lo[3], box_hi[3];
  int32_t dtype;                 /* storage format RBOS_F32 ... RBOS_BF16_XPAIR */
  double enc_scale, enc_offset;  /* eta - 1 = enc_offset + q / enc_scale; enc_scale > 0 */
  const void* field;             /* [dev] packed field from rbos_field_* (never modified) */
  /* pinhole camera: position, orthonormal forward/right/up, horizontal FOV (degrees) */
  double cam_pos[3], cam_fwd[3], cam_right[3], cam_up[3];
  double cam_fov_x_deg;
  int32_t width, height;
  const int32_t* pixel_ids;      /* [dev] optional pixel list (ids in [0, width*height)); NULL:
                                    every pixel */
  int32_t n_pixels;              /* length of pixel_ids, or width*height when NULL */
  /* back wall: a plane through wall_origin with unit normal wall_normal (facing the
     camera); (wall_u, wall_v) orthonormal in-plane axes defining wall coordinates */
  double wall_origin[3], wall_normal[3], wall_u[3], wall_v[3];
  int32_t wall_mode;             /* RBOS_WALL_PRINTED / RBOS_WALL_PROJECTOR */
  const float* pattern;          /* [dev] [pat_h][pat_w] luminance, row 0 at the top */
  int32_t pat_w, pat_h;
  double pat_extent_u, pat_extent_v;  /* printed: texture size on the wall, centred on
                                          wall_origin */
  double proj_pos[3], proj_fwd[3], proj_right[3], proj_up[3];  /* projector pinhole */
  double proj_fov_x_deg;
  /* integrator: Sharma RK4 step h in the ray parameter t (at most 4 voxels), step cap
     (1 .. 65536), checkpoint stride k (0 = no checkpoints; 1 = every step's state is
     stored and the adjoint reads it instead of replaying: 24 B per ray-step; 3 or 4: each
     segment is replayed once and the cell and fractions of its samples are kept on chip
     for the reverse, the fastest adjoint (3 is the autotuned choice on MI355X); 6:
     replayed in chunks of 6, whose smaller on-chip buffer lets more wavefronts share a
     compute unit; else a multiple of 8 up to 256, replayed in chunks of 8; any other
     value is rejected with RBOS_E_UNSUPPORTED; rbos_trace_adjoint needs k > 0).
     With the quasi-linear tracer the adjoint needs no states: any k > 0 stores only the
     per-ray header. */
  double step;
  int32_t max_steps;
  int32_t ckpt_stride;
  int32_t tracer;                /* RBOS_TRACER_NONLINEAR / RBOS_TRACER_QUASILINEAR; all scenes
                                    of one call share it */
  /* Eq. (2) pixel integral: spp rays per pixel (1 .. 1024; n_pixels * spp <= 2^30). With
     spp > 1, sample s of pixel p goes through the pixel centre plus the offset (ox, oy)
     (pixels; +y down the image): Philox-4x32-10 of the counter (p, s, 0, 0) under the key
     (seed, 0) gives words x0, x1, the uniforms u = (x >> 8) 2^-24, and each offset is the
     inverse CDF of the triangular density 1 - |x| on [-1, 1] at u. radiometry (0 or 1)
     weights each ray's radiance by |<n_w, v_w>| / |X_w - c|. */
  int32_t spp;
  uint32_t seed;
  int32_t radiometry;
} rbos_scene;

/* Per-scene forward outputs, indexed by ray r = s * n_pixels + i. */
typedef struct rbos_trace_out {
  float* wall_uv;    /* [dev] [n_rays][2] wall coordinates (u, v) of the hit, FP32-rounded */
  float* wall_duv;   /* [dev] [n_rays][2] (u, v) minus the undeflected camera ray's hit;
                        nullable */
  int32_t* n_steps;  /* [dev] [n_rays] Sharma steps taken inside the box */
  uint8_t* status;   /* [dev] [n_rays] RBOS_RAY_* bits */
  float* ckpt;       /* [dev] rbos_ckpt_bytes(scene) bytes of ray-state checkpoints,
                        written when scene.ckpt_stride > 0; opaque layout; must stay
                        unmodified until rbos_trace_adjoint has run */
  float* wall_dir;   /* [dev] [n_rays][3] unit ray direction at the wall (the camera ray's
                        for rays that miss the box; NaN for non-finite states); nullable,
                        but rbos_render needs it when scene.radiometry is set */
} rbos_trace_out;

/* Per-scene render inputs/outputs. */
typedef struct rbos_render_io {
  const float* target;  /* [dev] [n_pixels] measured image I_flow; nullable */
  float* image;         /* [dev] [n_pixels] rendered I(eta) */
  float* dL_duv;        /* [dev] [n_rays][2] dL_BOS/d(u, v) of each ray; needs target; nullable */
  float* loss;          /* [dev] one float: L_BOS of this scene; needs target; nullable */
  float* dL_ddir;       /* [dev] [n_rays][3] dL_BOS/d(wall_dir) of each ray (the radiometric
                           weight's dependence on the direction); needs target; required
                           with dL_duv when scene.radiometry is set, ignored otherwise */
} rbos_render_io;

/* Per-scene adjoint inputs/outputs. */
typedef struct rbos_adjoint_io {
  const float* dL_duv;  /* [dev] [n_rays][2] */
  double* grad;         /* [dev] [nz][ny][nx] FP64; the gradient w.r.t. eta - 1 is ADDED with
                           device-scope FP64 atomics that are correct only on coarse-grained
                           device memory (plain hipMalloc, a torch CUDA tensor); managed,
                           host-coherent or fine-grained buffers would accumulate wrong sums */
  const float* dL_ddir; /* [dev] [n_rays][3] dL/d(wall_dir); nullable (no direction term) */
} rbos_adjoint_io;

/* Launch shape (nullable: library defaults). */
typedef struct rbos_launch {
  int32_t tile_w, tile_h;     /* rays per wavefront tile, tile_w * tile_h == 64 */
  int32_t waves_per_block;    /* 1, 2 or 4 */
  int32_t persistent;         /* 1: persistent blocks pulling tiles from per-XCD queues */
  int32_t blocks_per_cu;      /* persistent mode: resident blocks per compute unit (1-16), or 0 for as
                                 many as each kernel's registers and LDS allow */
} rbos_launch;

/* Library and ABI version (RBOS_ABI_VERSION). */
int rbos_version(void);

/* Description of the last error on the calling thread ("" if none). The pointer stays
   valid until the thread's next rbos_* call. */
const char* rbos_last_error(void);

/* --- Sec. 2.A: field storage ------------------------------------------------------- */

/* Bytes of the packed field for nx*ny*nz voxels and a storage format (0 if invalid).
   Cell records (RBOS_F32, RBOS_F16, RBOS_BF16): one record per interpolation cell
   (i, j, k), i in [-1, nx-1] etc., i.e. (nx+1)(ny+1)(nz+1) records in x-fastest order
   starting at cell (-1, -1, -1), built from the cell's 8 corner codes q[a + 2b + 4c] at
   voxels (clamp(i+a), clamp(j+b), clamp(k+c)) (the apron cells repeat the edge voxels).
   FP16/BF16 records hold those 8 codes (16 B). FP32 records (32 B) hold the coefficients
   of the cell's trilinear polynomial in its fractions, q0, q1 - q0, q2 - q0,
   (q3 - q2) - (q1 - q0), q4 - q0, (q5 - q4) - (q1 - q0), (q6 - q4) - (q2 - q0),
   ((q7 - q6) - (q5 - q4)) - ((q3 - q2) - (q1 - q0)), each difference rounded to binary32
   in that order. X-pairs (*_XPAIR): (nx+1)(ny+2)(nz+2) entries (i, j, k), i in [-1, nx-1],
   j in [-1, ny], k in [-1, nz], x fastest, each holding the codes of voxels
   (clamp(i), clamp(j), clamp(k)) and (clamp(i+1), clamp(j), clamp(k)) (8 B FP32, 4 B
   for two 16-bit codes, low half first). */
size_t rbos_field_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t dtype);

/* Encode eta - 1 from temperature: delta = rho0G * (T0 / T) in binary32 (two correctly
   rounded operations), code q = RN_even((delta - c) * s) with c = (float)enc_offset and
   s = (float)enc_scale a power of two. T: [dev] [nz][ny][nx] kelvin. field: [dev]
   rbos_field_bytes() bytes. */
int rbos_field_from_temperature(int32_t nx, int32_t ny, int32_t nz, const float* T,
                                double rho0G, double T0, int32_t dtype, double enc_scale,
                                double enc_offset, void* field, void* stream);

/* Encode a given eta - 1 field: q = RN_even((delta - c) * s) as above.
   delta: [dev] [nz][ny][nx] FP32. */
int rbos_field_encode(int32_t nx, int32_t ny, int32_t nz, const float* delta, int32_t dtype,
                      double enc_scale, double enc_offset, void* field, void* stream);

/* Code scale for 16-bit storage (Sec. 2.A: the stored quantity is eta - 1): the largest
   power of two s with s * max |eta - 1 - enc_offset| <= 2^14 over eta - 1 in
   [delta_lo, delta_hi], so the codes neither overflow nor (for FP16) fall into the
   subnormal range; 1 for RBOS_F32. Returns 0 for an unknown dtype or an invalid range.
   The offset that makes 16-bit storage accurate is the ambient eta - 1 (rho0 G at
   T = T0): the codes then hold only the perturbation. */
double rbos_code_scale(int32_t dtype, double delta_lo, double delta_hi, double enc_offset);

/* The same for a temperature field with T in [T_lo, T_hi] kelvin (T_lo > 0):
   eta - 1 = rho0G T0 / T spans [rho0G T0 / T_hi, rho0G T0 / T_lo]. */
double rbos_code_scale_temperature(int32_t dtype, double T_lo, double T_hi, double rho0G, double T0,
                                   double enc_offset);

/* --- Sec. 2.B / 2.C / 2.D: tracing, rendering, gradient ----------------------------- */

/* Bytes of the checkpoint buffer of one scene (0 when ckpt_stride == 0). */
size_t rbos_ckpt_bytes(const rbos_scene* scene);

/* Bytes of device workspace needed by rbos_trace_forward / rbos_render /
   rbos_trace_adjoint for this set of scenes (scene table, queue counters, loss
   partials, the persistent adjoint's per-tile step counts and tile order). One
   workspace may serve all three calls in stream order. */
size_t rbos_workspace_bytes(const rbos_scene* scenes, int32_t n_scenes);

/* Trace every ray of every scene (Eq. 1 with Sharma steps) to the back wall; one launch
   for all scenes. scenes, outs: host arrays of n_scenes entries. launch: nullable.
   Writes outs[s] arrays; with ckpt_stride > 0 also the checkpoints. */
int rbos_trace_forward(const rbos_scene* scenes, int32_t n_scenes, const rbos_trace_out* outs,
                       const rbos_launch* launch, void* workspace, size_t ws_bytes, void* stream);

/* Render the traced hits (wall luminance, bilinear, times the radiometric weight when
   set) and average each pixel's rays; with a target, the residual, L_BOS per scene
   (deterministic FP32 reduction) and per ray dL_BOS/d(u, v) (and dL_BOS/d(wall_dir)).
   Also sets RBOS_RAY_OFF_PATTERN in outs[s].status. */
int rbos_render(const rbos_scene* scenes, int32_t n_scenes, const rbos_trace_out* outs,
                const rbos_render_io* io, void* workspace, size_t ws_bytes, void* stream);

/* Back-propagate dL/d(u, v) (and dL/d(wall_dir)) per ray through the wall step and
   every Sharma step (replayed from the forward checkpoints) to dL/d(eta - 1) per voxel,
   accumulated in FP64 into io[s].grad. Needs the same scenes (ckpt_stride > 0), the
   forward outputs and the unmodified field. A persistent launch first orders the tiles
   by the forward's step counts (longest first); the order changes only the order of
   the FP64 additions. */
int rbos_trace_adjoint(const rbos_scene* scenes, int32_t n_scenes, const rbos_trace_out* outs,
                       const rbos_adjoint_io* io, const rbos_launch* launch, void* workspace,
                       size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph capture, tight
   serving loops, harnesses that forbid hipMalloc): rbos_trace_adjoint without a
   workspace argument. Same arguments, results and errors otherwise. The scene table,
   queue counters, per-tile step counts and tile order live in a static device array of
   RBOS_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on until the
   process ends (its address is looked up once per device, on the first call with that
   device current). Calls whose scenes need more than that (rbos_workspace_bytes-sized
   layout for the given launch) return RBOS_E_WORKSPACE before anything is enqueued. The
   array is shared by every call on one device and keeps the last call's contents (each
   call re-initialises what it reads): calls that overlap in time on one device, on any
   streams or threads, race and must be serialised by the caller. No device memory is
   allocated or freed. */
#define RBOS_NOALLOC_SCRATCH_BYTES (4u << 20)
int rbos_trace_adjoint_noalloc(const rbos_scene* scenes, int32_t n_scenes, const rbos_trace_out* outs,
                               const rbos_adjoint_io* io, const rbos_launch* launch, void* stream);

/* --- Sec. 2.D: the network field ---------------------------------------------------- */

/* The temperature, pressure and velocity are one MLP of the position (Sec. 2.D):
   (T_nd, p, u_x, u_y, u_z) = MLP(xhat), xhat = 2 (x - box_lo) / (box_hi - box_lo) - 1,
   with `depth` hidden layers of `width` tanh units and a linear output layer, and
   T = T0 + (T_in - T0) T_nd. The parameters are packed per layer (3 -> width,
   width -> width repeated depth - 1 times, width -> 5): the weights [in][out] row-major,
   then the biases [out]. FP32 throughout; the hidden layers run on the matrix cores. */
typedef struct rbos_mlp {
  int32_t width;             /* hidden units per layer: 64 */
  int32_t depth;             /* hidden layers: 1 .. 8 */
  const float* params;       /* [dev] rbos_mlp_param_count(width, depth) floats */
  double box_lo[3], box_hi[3];  /* normalisation box of the inputs (finite, lo < hi) */
} rbos_mlp;

/* Number of packed parameters (0 if width or depth is unsupported). */
size_t rbos_mlp_param_count(int32_t width, int32_t depth);

/* Workspace bytes for one point set of n_points: the activations kept by
   rbos_mlp_forward for a following rbos_mlp_backward, and reduction buffers. */
size_t rbos_mlp_workspace_bytes(int32_t width, int32_t depth, int64_t n_points);

/* Evaluate the MLP at n_points points: points [dev] [n][3] in metres, or NULL for the
   voxel centres of the grid grid_dims (host int32[3] = nx, ny, nz over the MLP box,
   x fastest; n_points must be nx*ny*nz). Writes out [dev] [n][5] and/or
   T [dev] [n] = T0 + (T_in - T0) out_0 (each nullable) and keeps the activations in the
   workspace (256-byte aligned, >= rbos_mlp_workspace_bytes). */
int rbos_mlp_forward(const rbos_mlp* mlp, const float* points, int64_t n_points, const int32_t* grid_dims,
                     float* out, float* T, double T0, double T_in, void* workspace, size_t ws_bytes, void* stream);

/* Parameter gradient of a loss given per point as dL_dout [dev] [n][5]: ADDS
   sum_i dL_dout_i . d out_i / d params into dparams [dev] (param_count floats). Needs the
   workspace of an rbos_mlp_forward on the same points and parameters, unmodified since;
   the block sums are reduced in a fixed order (deterministic). */
int rbos_mlp_backward(const rbos_mlp* mlp, const float* points, int64_t n_points, const int32_t* grid_dims,
                      const float* dL_dout, float* dparams, void* workspace, size_t ws_bytes, void* stream);

/* Chain of the BOS loss to the network (Sec. 2.A, 2.D): from dL/d(eta - 1) per voxel
   (grad_delta [dev] FP64, the adjoint's output) and the voxel temperatures T [dev] [n]
   (kelvin, > 0), writes dL_dout [dev] [n][5] with channel 0 =
   grad_delta * (-rho0G T0 / T^2) * (T_in - T0) and channels 1..4 = 0. */
int rbos_mlp_bos_seed(int64_t n, const float* T, const double* grad_delta, double rho0G, double T0, double T_in,
                      float* dL_dout, void* stream);

/* Boundary loss (Sec. 2.D): L_Gamma = sum_i sum_k ((out_ik - target_ik) / norm_k)^2 over
   n points, each field divided by its normaliser (norms: host double[5] > 0, one per
   output; the paper divides each field by its maximum value). Writes the seed
   dL_dout [dev] [n][5] = 2 (out - target) / norm^2 for rbos_mlp_backward and, if loss
   [dev] (one float) is given, L_Gamma, summed in a fixed order in the workspace
   (>= rbos_mlp_fit_workspace_bytes(n), 256-byte aligned). */
size_t rbos_mlp_fit_workspace_bytes(int64_t n_points);
int rbos_mlp_fit_seed(int64_t n, const float* out, const float* target, const double* norms, float* dL_dout,
                      float* loss, void* workspace, size_t ws_bytes, void* stream);

/* Physics-informed loss (Sec. 2.D): at n collocation points x (metres),
   L_PDE = sum_i g1 r_mass^2 + g2 |r_mom|^2 + g3 r_heat^2 with the Boussinesq residuals in
   nondimensional coordinates x_nd = x / L and gravity along -z:
     r_mass = div u,  r_mom = (u . grad) u + grad p - lap(u) / Re + Ri T_nd e_g,
     r_heat = (u . grad) T_nd - lap(T_nd) / Pe.
   The derivatives come from forward-mode jets of the MLP (value, first and second
   derivative along each axis, 7 channels per point, the hidden layers on the matrix
   cores); the parameter gradient from their reverse. */
typedef struct rbos_pde {
  double Re, Pe, Ri;   /* Reynolds, Peclet and Richardson numbers (Re, Pe > 0) */
  double L;            /* characteristic length in metres (> 0) */
  double gamma[3];     /* weights of the mass, momentum and heat residuals */
} rbos_pde;

/* Workspace bytes of rbos_mlp_pde_loss for n_points collocation points. */
size_t rbos_mlp_pde_workspace_bytes(int32_t width, int32_t depth, int64_t n_points);

/* Residuals, loss and parameter gradient at the collocation points [dev] [n][3]. Writes
   residuals [dev] [n][5] (r_mass, r_mom x 3, r_heat) and loss [dev] (one float, summed in
   a fixed order) when given, and ADDS dL_PDE/d params into dparams [dev] when given. */
int rbos_mlp_pde_loss(const rbos_mlp* mlp, const rbos_pde* pde, const float* points, int64_t n_points, float* loss,
                      float* dparams, float* residuals, void* workspace, size_t ws_bytes, void* stream);

/* --- binding support --------------------------------------------------------------- */

/* Layout of the public structs for binding checks: which = 0 rbos_scene,
   1 rbos_trace_out, 2 rbos_render_io, 3 rbos_adjoint_io, 4 rbos_launch, 5 rbos_mlp,
   6 rbos_pde. Writes up to
   max_fields member offsets (declaration order) and returns sizeof, or 0 if unknown. */
size_t rbos_struct_layout(int32_t which, size_t* offsets, int32_t max_fields);

#ifdef __cplusplus
}
#endif
#endif /* RBOS_H */
