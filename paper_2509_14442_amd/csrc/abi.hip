// abi.hip -- the C ABI of librbos: host-side validation, device scene tables and the
// launches of the field, forward, render and adjoint kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rbos.h"
#include "rbos_device.hpp"
#include "rbos_launch.hpp"
#include "mlp_launch.hpp"

namespace {

using rbos::df;
using rbos::SceneDev;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

df to_df(double x) {
  float hi = (float)x;
  float lo = (float)(x - (double)hi);
  return {hi, lo};
}

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }
double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
bool unit3(const double* v) { return finite3(v) && std::fabs(dot3(v, v) - 1.0) < 1e-9; }
bool orthonormal(const double* a, const double* b, const double* c) {
  return unit3(a) && unit3(b) && unit3(c) && std::fabs(dot3(a, b)) < 1e-9 && std::fabs(dot3(a, c)) < 1e-9 &&
         std::fabs(dot3(b, c)) < 1e-9;
}
bool pow2(double s) {
  if (!(s > 0.0) || !std::isfinite(s)) return false;
  int e;
  return std::frexp(s, &e) == 0.5;
}

struct Launch {
  int tile_w = 8, tile_h = 8, wpb = 4, persistent = 0, blocks_per_cu = 0;
};

int check_launch(const rbos_launch* L, Launch& out) {
  if (!L) return RBOS_OK;
  if (L->tile_w < 1 || L->tile_h < 1 || L->tile_w * L->tile_h != 64 || (L->tile_w & (L->tile_w - 1)))
    return fail(RBOS_E_RANGE, "launch: tile_w * tile_h must be 64 with tile_w a power of two (got %d x %d)",
                L->tile_w, L->tile_h);
  if (L->waves_per_block != 1 && L->waves_per_block != 2 && L->waves_per_block != 4)
    return fail(RBOS_E_RANGE, "launch: waves_per_block must be 1, 2 or 4 (got %d)", L->waves_per_block);
  if (L->persistent != 0 && L->persistent != 1) return fail(RBOS_E_RANGE, "launch: persistent must be 0 or 1");
  if (L->persistent && (L->blocks_per_cu < 0 || L->blocks_per_cu > 16))
    return fail(RBOS_E_RANGE, "launch: blocks_per_cu must be in [0, 16] (got %d)", L->blocks_per_cu);
  out.tile_w = L->tile_w;
  out.tile_h = L->tile_h;
  out.wpb = L->waves_per_block;
  out.persistent = L->persistent;
  out.blocks_per_cu = L->blocks_per_cu;
  return RBOS_OK;
}

bool valid_dtype(int32_t dtype) { return dtype >= RBOS_F32 && dtype <= RBOS_BF16_XPAIR; }

int check_scene(const rbos_scene* S, int idx, bool need_render) {
  if (S->nx < 2 || S->ny < 2 || S->nz < 2 || S->nx > RBOS_MAX_DIM || S->ny > RBOS_MAX_DIM || S->nz > RBOS_MAX_DIM)
    return fail(RBOS_E_SHAPE, "scene %d: voxel counts must be in [2, %d] (got %d x %d x %d)", idx, RBOS_MAX_DIM, S->nx,
                S->ny, S->nz);
  if (!finite3(S->box_lo) || !finite3(S->box_hi) || !(S->box_lo[0] < S->box_hi[0]) ||
      !(S->box_lo[1] < S->box_hi[1]) || !(S->box_lo[2] < S->box_hi[2]))
    return fail(RBOS_E_RANGE, "scene %d: box must be finite with lo < hi on every axis", idx);
  if (!valid_dtype(S->dtype)) return fail(RBOS_E_DTYPE, "scene %d: unknown dtype %d", idx, S->dtype);
  if (!pow2(S->enc_scale)) return fail(RBOS_E_RANGE, "scene %d: enc_scale must be a positive power of two", idx);
  if (!std::isfinite(S->enc_offset)) return fail(RBOS_E_RANGE, "scene %d: enc_offset must be finite", idx);
  if (!S->field) return fail(RBOS_E_NULL, "scene %d: field is NULL", idx);
  if (!finite3(S->cam_pos) || !orthonormal(S->cam_fwd, S->cam_right, S->cam_up))
    return fail(RBOS_E_RANGE, "scene %d: camera position must be finite and fwd/right/up orthonormal", idx);
  if (!(S->cam_fov_x_deg > 0.0 && S->cam_fov_x_deg < 179.0))
    return fail(RBOS_E_RANGE, "scene %d: cam_fov_x_deg must be in (0, 179)", idx);
  if (S->width < 1 || S->height < 1 || (long long)S->width * S->height > (1LL << 30))
    return fail(RBOS_E_SHAPE, "scene %d: width and height must be >= 1 with width*height <= 2^30", idx);
  if (!S->pixel_ids && (long long)S->n_pixels != (long long)S->width * S->height)
    return fail(RBOS_E_SHAPE, "scene %d: n_pixels must equal width*height when pixel_ids is NULL", idx);
  if (S->n_pixels < 0) return fail(RBOS_E_SHAPE, "scene %d: n_pixels < 0", idx);
  if (S->spp < 1 || S->spp > 1024) return fail(RBOS_E_RANGE, "scene %d: spp must be in [1, 1024] (got %d)", idx, S->spp);
  if ((long long)S->n_pixels * S->spp > (1LL << 30))
    return fail(RBOS_E_SHAPE, "scene %d: n_pixels * spp must be <= 2^30", idx);
  if (S->radiometry != 0 && S->radiometry != 1)
    return fail(RBOS_E_RANGE, "scene %d: radiometry must be 0 or 1", idx);
  if (!finite3(S->wall_origin) || !orthonormal(S->wall_normal, S->wall_u, S->wall_v))
    return fail(RBOS_E_RANGE, "scene %d: wall origin must be finite and normal/u/v orthonormal", idx);
  if (S->wall_mode != RBOS_WALL_PRINTED && S->wall_mode != RBOS_WALL_PROJECTOR)
    return fail(RBOS_E_RANGE, "scene %d: unknown wall_mode %d", idx, S->wall_mode);
  double vmin = 1e300;
  for (int a = 0; a < 3; ++a) {
    int n = a == 0 ? S->nx : (a == 1 ? S->ny : S->nz);
    vmin = std::fmin(vmin, (S->box_hi[a] - S->box_lo[a]) / n);
  }
  if (!(S->step > 0.0) || !std::isfinite(S->step) || S->step > 4.0 * vmin)
    return fail(RBOS_E_RANGE, "scene %d: step must be in (0, 4 * smallest voxel]", idx);
  if (S->max_steps < 1 || S->max_steps > (1 << 16))
    return fail(RBOS_E_RANGE, "scene %d: max_steps must be in [1, 65536]", idx);
  if (S->tracer != RBOS_TRACER_NONLINEAR && S->tracer != RBOS_TRACER_QUASILINEAR)
    return fail(RBOS_E_RANGE, "scene %d: tracer must be RBOS_TRACER_NONLINEAR or RBOS_TRACER_QUASILINEAR", idx);
  if (S->ckpt_stride != 0 && S->ckpt_stride != 1 && S->ckpt_stride != 3 && S->ckpt_stride != 4 &&
      S->ckpt_stride != 6 && !(S->ckpt_stride % 8 == 0 && S->ckpt_stride <= 256 && S->ckpt_stride > 0))
    return fail(RBOS_E_UNSUPPORTED,
                "scene %d: ckpt_stride must be 0, 1, 3, 4, 6 or a multiple of 8 up to 256 (got %d)", idx,
                S->ckpt_stride);
  if (need_render) {
    if (!S->pattern) return fail(RBOS_E_NULL, "scene %d: pattern is NULL", idx);
    if (S->pat_w < 1 || S->pat_h < 1 || S->pat_w > (1 << 15) || S->pat_h > (1 << 15))
      return fail(RBOS_E_SHAPE, "scene %d: pattern size must be in [1, 32768]", idx);
    if (S->wall_mode == RBOS_WALL_PRINTED && !(S->pat_extent_u > 0.0 && S->pat_extent_v > 0.0 &&
                                               std::isfinite(S->pat_extent_u) && std::isfinite(S->pat_extent_v)))
      return fail(RBOS_E_RANGE, "scene %d: printed pattern extents must be positive", idx);
    if (S->wall_mode == RBOS_WALL_PROJECTOR &&
        (!finite3(S->proj_pos) || !orthonormal(S->proj_fwd, S->proj_right, S->proj_up) ||
         !(S->proj_fov_x_deg > 0.0 && S->proj_fov_x_deg < 179.0)))
      return fail(RBOS_E_RANGE, "scene %d: projector pose must be orthonormal with fov in (0, 179)", idx);
  }
  return RBOS_OK;
}

// tiles of one sample plane (the scene has spp planes)
long long tiles_per_plane(const rbos_scene* S, const Launch& L, int* tiles_x) {
  if (S->pixel_ids) {
    *tiles_x = 0;
    return ((long long)S->n_pixels + 63) / 64;
  }
  int tx = (S->width + L.tile_w - 1) / L.tile_w;
  int ty = (S->height + L.tile_h - 1) / L.tile_h;
  *tiles_x = tx;
  return (long long)tx * ty;
}

long long tiles_of(const rbos_scene* S, const Launch& L, int* tiles_x) {
  return tiles_per_plane(S, L, tiles_x) * (S->spp > 0 ? S->spp : 1);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// checkpoint slots per ray: states at steps k, 2k, ... below max_steps; the quasi-linear
// adjoint needs only the ray header
int ckpt_slots(const rbos_scene* S) {
  if (S->ckpt_stride <= 0 || S->tracer == RBOS_TRACER_QUASILINEAR) return 0;
  return (S->max_steps - 1) / S->ckpt_stride;
}

// entries per checkpoint component and sample plane: the image in 8 x 8 pixel blocks
long long ckpt_plane_entries(const rbos_scene* S) {
  return (long long)((S->width + 7) / 8) * ((S->height + 7) / 8) * 64;
}

// entries per checkpoint component: spp image planes, or the ray list (all samples)
// rounded up to 64
long long ckpt_entries(const rbos_scene* S) {
  const long long spp = S->spp > 0 ? S->spp : 1;
  if (S->pixel_ids) return ((long long)S->n_pixels * spp + 63) / 64 * 64;
  return ckpt_plane_entries(S) * spp;
}

struct Layout {
  size_t table, queues, partials, tile_cost, tile_order, total;
  long long total_tiles;
  int total_render_blocks;
};

Layout layout(const rbos_scene* scenes, int n, const Launch& L) {
  Layout y{};
  y.table = 0;
  y.queues = align256(sizeof(SceneDev) * (size_t)n);
  y.partials = y.queues + 256;
  long long tiles = 0;
  long long rblocks = 0;
  for (int i = 0; i < n; ++i) {
    int tx;
    tiles += tiles_of(&scenes[i], L, &tx);
    rblocks += ((long long)scenes[i].n_pixels + 255) / 256;
  }
  y.total_tiles = tiles;
  y.total_render_blocks = (int)rblocks;
  y.tile_cost = align256(y.partials + sizeof(float) * (size_t)(rblocks > 0 ? rblocks : 1));
  y.tile_order = align256(y.tile_cost + sizeof(int) * (size_t)(tiles > 0 ? tiles : 1));
  y.total = align256(y.tile_order + sizeof(int) * (size_t)(tiles > 0 ? tiles : 1));
  return y;
}

// Reciprocal for dividing record indices r < 2^27 by d (1 <= d < 2^18): with
// L = ceil(log2 d), k = 27 + L and m = ceil(2^k / d), floor(r / d) = (r * m) >> k, because
// m d - 2^k < d makes the added error r (m d - 2^k) / (d 2^k) < 2^27 / 2^k <= 1 / d, less
// than the gap to the next integer; m < 2^28 + 1 keeps r * m below 2^56.
void rec_divisor(int d, unsigned& m, int& k) {
  int L = 0;
  while ((1 << L) < d) ++L;
  k = 27 + L;
  m = (unsigned)(((1ull << k) + (unsigned long long)d - 1) / (unsigned long long)d);
}

SceneDev make_dev(const rbos_scene* S, const Launch& L, int tile_begin, int render_block_begin) {
  SceneDev d;
  std::memset(&d, 0, sizeof d);
  const int n[3] = {S->nx, S->ny, S->nz};
  const double scale = S->enc_scale;
  const double dec = 1.0 / scale;
  for (int a = 0; a < 3; ++a) {
    d.n[a] = n[a];
    double vox = (S->box_hi[a] - S->box_lo[a]) / n[a];
    d.km[a] = (float)(dec / (vox * vox));
    d.vox[a] = (float)vox;
    d.lo_f[a] = (float)S->box_lo[a];
    d.hi_bound[a] = (float)n[a] + 0.5f;
    d.n_f[a] = (float)n[a];
    d.lo[a] = to_df(S->box_lo[a]);
    d.hi[a] = to_df(S->box_hi[a]);
    d.inv_vox[a] = to_df(1.0 / vox);
    d.cam_pos[a] = to_df(S->cam_pos[a]);
    d.cam_fwd[a] = to_df(S->cam_fwd[a]);
    d.cam_right[a] = to_df(S->cam_right[a]);
    d.cam_up[a] = to_df(S->cam_up[a]);
    d.wall_org[a] = to_df(S->wall_origin[a]);
    d.wall_n[a] = to_df(S->wall_normal[a]);
    d.wall_u[a] = to_df(S->wall_u[a]);
    d.wall_v[a] = to_df(S->wall_v[a]);
    d.wall_org_f[a] = (float)S->wall_origin[a];
    d.wall_n_f[a] = (float)S->wall_normal[a];
    d.wall_u_f[a] = (float)S->wall_u[a];
    d.wall_v_f[a] = (float)S->wall_v[a];
    d.proj_pos[a] = to_df(S->proj_pos[a]);
    d.proj_fwd[a] = to_df(S->proj_fwd[a]);
    d.proj_right[a] = to_df(S->proj_right[a]);
    d.proj_up[a] = to_df(S->proj_up[a]);
  }
  // record strides of the padded cell grid, or entry strides of the x-pair array (one
  // more row and plane in y and z)
  d.P1 = rbos::is_xpair(S->dtype) ? S->ny + 2 : S->ny + 1;
  d.P0 = S->nx + 1;
  d.P01 = d.P0 * d.P1;
  rec_divisor(d.P0, d.rec_div_m[0], d.rec_div_s[0]);
  rec_divisor(d.P01, d.rec_div_m[1], d.rec_div_s[1]);
  d.dtype = S->dtype;
  d.field = S->field;
  d.dec = (float)dec;
  d.inv_dec = (float)scale;
  d.inv_dec_d = 1.0 / (double)d.dec;
  d.off = (float)S->enc_offset;
  d.one_plus_off = (float)(1.0 + (double)(float)S->enc_offset);
  const double h = S->step;
  d.h = to_df(h);
  d.hf = (float)h;
  d.h_2 = (float)(h / 2.0);
  d.h_6 = (float)(h / 6.0);
  d.h2_8 = (float)(h * h / 8.0);
  d.h2_2 = (float)(h * h / 2.0);
  d.h2_6 = (float)(h * h / 6.0);
  for (int a = 0; a < 3; ++a) {
    const double vox = (S->box_hi[a] - S->box_lo[a]) / n[a];
    const double km = dec / (vox * vox);
    d.c_p2[a] = (float)(h * h / 8.0 * km);
    d.c_p3[a] = (float)(h * h / 2.0 * km);
    d.c_x[a] = (float)(h * h / 6.0 * km);
    d.c_v[a] = (float)(h / 6.0 * km);
    d.c_x2[a] = 2.0f * d.c_x[a];
    d.c_v4[a] = 4.0f * d.c_v[a];
  }
  d.max_steps = S->max_steps;
  d.ckpt_k = S->ckpt_stride > 0 ? S->ckpt_stride : 1;
  d.ckpt_slots = ckpt_slots(S);
  d.tracer = S->tracer;
  const double t = std::tan(0.5 * S->cam_fov_x_deg * M_PI / 180.0);
  d.cam_ax = to_df(t / S->width);
  d.cam_cx = to_df(t);
  d.cam_cy = to_df(t * S->height / S->width);
  d.width = S->width;
  d.height = S->height;
  d.pixel_ids = S->pixel_ids;
  d.n_pix = S->n_pixels;
  d.spp = S->spp;
  d.n_rays = S->n_pixels * S->spp;
  d.seed = S->seed;
  d.radiometry = S->radiometry;
  int tx;
  d.tiles_plane = (int)tiles_per_plane(S, L, &tx);
  long long nt = tiles_of(S, L, &tx);
  d.tile_w = L.tile_w;
  d.tile_h = L.tile_h;
  d.tiles_x = tx;
  d.n_tiles = (int)nt;
  d.tile_begin = tile_begin;
  d.ckpt_pad = ckpt_entries(S);
  d.ckpt_plane = ckpt_plane_entries(S);
  d.ckpt_tx = (S->width + 7) / 8;
  d.wall_mode = S->wall_mode;
  d.pattern = S->pattern;
  d.pat_w = S->pat_w;
  d.pat_h = S->pat_h;
  if (S->wall_mode == RBOS_WALL_PRINTED && S->pat_extent_u > 0 && S->pat_extent_v > 0) {
    d.pat_half_u = to_df(0.5 * S->pat_extent_u);
    d.pat_half_v = to_df(0.5 * S->pat_extent_v);
    d.pat_inv_tu = to_df(S->pat_w / S->pat_extent_u);
    d.pat_inv_tv = to_df(S->pat_h / S->pat_extent_v);
  }
  if (S->proj_fov_x_deg > 0 && S->pat_w > 0) {
    const double tp = std::tan(0.5 * S->proj_fov_x_deg * M_PI / 180.0);
    d.proj_inv_tx = to_df(1.0 / tp);
    d.proj_inv_ty = to_df(1.0 / (tp * S->pat_h / S->pat_w));
  }
  d.render_block_begin = render_block_begin;
  d.render_blocks = (int)(((long long)S->n_pixels + 255) / 256);
  return d;
}

// Common front half of the three tracing entry points.
struct Prepared {
  Launch L;
  Layout Y;
  std::vector<SceneDev> table;
};

int prepare(const rbos_scene* scenes, int32_t n_scenes, const rbos_launch* launch, void* workspace, size_t ws_bytes,
            bool need_render, Prepared& P) {
  if (!scenes) return fail(RBOS_E_NULL, "scenes is NULL");
  if (n_scenes < 0) return fail(RBOS_E_SHAPE, "n_scenes < 0");
  int rc = check_launch(launch, P.L);
  if (rc) return rc;
  for (int i = 0; i < n_scenes; ++i) {
    rc = check_scene(&scenes[i], i, need_render);
    if (rc) return rc;
    if (ckpt_entries(&scenes[i]) > (1LL << 31) - 1)
      return fail(RBOS_E_SHAPE, "scene %d: too many checkpoint entries (8 x 8 blocks times spp)", i);
    if (scenes[i].dtype != scenes[0].dtype)
      return fail(RBOS_E_UNSUPPORTED, "scene %d: all scenes of one call must share the storage dtype", i);
    if (scenes[i].tracer != scenes[0].tracer)
      return fail(RBOS_E_UNSUPPORTED, "scene %d: all scenes of one call must share the tracer", i);
  }
  P.Y = layout(scenes, n_scenes, P.L);
  if (P.Y.total_tiles > (1LL << 30)) return fail(RBOS_E_SHAPE, "too many rays in one call");
  if (n_scenes > 0) {
    if (!workspace) return fail(RBOS_E_WORKSPACE, "workspace is NULL");
    if (ws_bytes < P.Y.total) return fail(RBOS_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, P.Y.total);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
      return fail(RBOS_E_WORKSPACE, "workspace must be 256-byte aligned");
  }
  P.table.resize((size_t)n_scenes);
  int tile = 0, rblk = 0;
  for (int i = 0; i < n_scenes; ++i) {
    P.table[i] = make_dev(&scenes[i], P.L, tile, rblk);
    tile += P.table[i].n_tiles;
    rblk += P.table[i].render_blocks;
  }
  return RBOS_OK;
}

// compute units of the current device, queried once per device (safe from any thread)
int compute_units() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cache[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

int finish_launch(Prepared& P, void* workspace, hipStream_t stream, rbos::LaunchPlan& plan) {
  unsigned char* ws = static_cast<unsigned char*>(workspace);
  hipError_t e = rbos::launch_upload(ws + P.Y.table, P.table.data(), sizeof(SceneDev) * P.table.size(), stream);
  if (e != hipSuccess) return fail(RBOS_E_HIP, "scene table upload failed: %s", hipGetErrorString(e));
  plan.scenes = reinterpret_cast<const SceneDev*>(ws + P.Y.table);
  plan.n_scenes = (int)P.table.size();
  plan.total_tiles = (int)P.Y.total_tiles;
  plan.wpb = P.L.wpb;
  plan.dtype = P.table.empty() ? 0 : P.table[0].dtype;
  plan.persistent = P.L.persistent;
  plan.blocks_per_cu = P.L.blocks_per_cu;
  plan.n_cus = compute_units();
  plan.queues = reinterpret_cast<unsigned int*>(ws + P.Y.queues);
  plan.total_render_blocks = P.Y.total_render_blocks;
  plan.partials = reinterpret_cast<float*>(ws + P.Y.partials);
  plan.tile_cost = reinterpret_cast<int*>(ws + P.Y.tile_cost);
  plan.tile_order = reinterpret_cast<int*>(ws + P.Y.tile_order);
  int longest = 1;
  for (const SceneDev& d : P.table) longest = std::max(longest, d.max_steps);
  plan.order_shift = 0;
  while ((longest >> plan.order_shift) >= 1024) ++plan.order_shift;
  plan.ckpt_k = P.table.empty() ? 0 : P.table[0].ckpt_k;
  plan.tracer = P.table.empty() ? 0 : P.table[0].tracer;
  if (P.L.persistent) {
    e = rbos::launch_fill_u32(plan.queues, 0u, 16, stream);
    if (e != hipSuccess) return fail(RBOS_E_HIP, "queue reset failed: %s", hipGetErrorString(e));
  }
  return RBOS_OK;
}

// Per-scene arguments of the two adjoint entry points, checked and bound into the scene
// table (host only).
int adjoint_bind(Prepared& P, const rbos_scene* scenes, int32_t n_scenes, const rbos_trace_out* outs,
                 const rbos_adjoint_io* io) {
  if (n_scenes > 0 && (!outs || !io)) return fail(RBOS_E_NULL, "outs or io is NULL");
  for (int i = 0; i < n_scenes; ++i) {
    if (scenes[i].ckpt_stride <= 0) return fail(RBOS_E_UNSUPPORTED, "scene %d: the adjoint needs ckpt_stride > 0", i);
    if (scenes[i].ckpt_stride != scenes[0].ckpt_stride)
      return fail(RBOS_E_UNSUPPORTED, "scene %d: all scenes of one adjoint call must share ckpt_stride", i);
    const bool rays = scenes[i].n_pixels > 0;
    if (rays && (!outs[i].ckpt || !outs[i].n_steps || !outs[i].status))
      return fail(RBOS_E_NULL, "scene %d: ckpt, n_steps and status are required", i);
    if (rays && !io[i].dL_duv) return fail(RBOS_E_NULL, "scene %d: dL_duv is required", i);
    if (!io[i].grad) return fail(RBOS_E_NULL, "scene %d: grad is required", i);
    SceneDev& d = P.table[i];
    d.n_steps = outs[i].n_steps;
    d.status = outs[i].status;
    d.ckpt = outs[i].ckpt;
    d.adj_dL_duv = io[i].dL_duv;
    d.adj_dL_ddir = io[i].dL_ddir;
    d.grad = io[i].grad;
  }
  return RBOS_OK;
}

// Enqueue the adjoint: scene table upload into `ws` (the caller's workspace or the
// static scratch), tile order, adjoint kernel.
int adjoint_enqueue(Prepared& P, int32_t n_scenes, void* ws, hipStream_t stream_h) {
  if (n_scenes == 0 || P.Y.total_tiles == 0) return RBOS_OK;
  rbos::LaunchPlan plan{};
  int rc = finish_launch(P, ws, stream_h, plan);
  if (rc) return rc;
  hipError_t e = hipSuccess;
  if (plan.persistent) {
    e = rbos::launch_tile_order(plan, stream_h);
    if (e != hipSuccess) return fail(RBOS_E_HIP, "tile order launch failed: %s", hipGetErrorString(e));
  }
  e = rbos::launch_trace_adj(plan, stream_h);
  if (e != hipSuccess) return fail(RBOS_E_HIP, "adjoint launch failed: %s", hipGetErrorString(e));
  return RBOS_OK;
}

// Device scratch of rbos_trace_adjoint_noalloc (scene table, queue counters, per-tile
// step counts and tile order), for callers that cannot allocate. Each device holds its
// own copy at its own address: host code takes that address from hipGetSymbolAddress,
// once per device, and never uses the array's name as a device pointer.
constexpr size_t NOALLOC_SCRATCH_BYTES = RBOS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

// Device address of `scratch` on the current device, looked up on the first call per
// device (with that device current) and kept.
int noalloc_scratch(void** out) {
  static std::mutex mu;
  static void* addr[MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(RBOS_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(RBOS_E_UNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RBOS_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    addr[dev] = p;
  }
  *out = addr[dev];
  return RBOS_OK;
}

}  // namespace

extern "C" {

int rbos_version(void) { return RBOS_ABI_VERSION; }

const char* rbos_last_error(void) { return g_err.c_str(); }

size_t rbos_field_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t dtype) {
  if (nx < 2 || ny < 2 || nz < 2 || nx > RBOS_MAX_DIM || ny > RBOS_MAX_DIM || nz > RBOS_MAX_DIM) return 0;
  if (!valid_dtype(dtype)) return 0;
  const bool f32 = rbos::code_type(dtype) == rbos::DT_F32;
  if (rbos::is_xpair(dtype))
    return (f32 ? 8 : 4) * (size_t)(nx + 1) * (size_t)(ny + 2) * (size_t)(nz + 2);
  return (f32 ? 32 : 16) * (size_t)(nx + 1) * (size_t)(ny + 1) * (size_t)(nz + 1);
}

static int field_common(int32_t nx, int32_t ny, int32_t nz, const float* src, int from_t, double rho0G, double T0,
                        int32_t dtype, double scale, double offset, void* field, void* stream) {
  g_err.clear();
  if (nx < 2 || ny < 2 || nz < 2 || nx > RBOS_MAX_DIM || ny > RBOS_MAX_DIM || nz > RBOS_MAX_DIM)
    return fail(RBOS_E_SHAPE, "voxel counts must be in [2, %d]", RBOS_MAX_DIM);
  if (!valid_dtype(dtype)) return fail(RBOS_E_DTYPE, "unknown dtype %d", dtype);
  if (!src || !field) return fail(RBOS_E_NULL, "input or field pointer is NULL");
  if (!pow2(scale)) return fail(RBOS_E_RANGE, "enc_scale must be a positive power of two");
  if (!std::isfinite(offset)) return fail(RBOS_E_RANGE, "enc_offset must be finite");
  if (from_t && (!(rho0G > 0.0) || !std::isfinite(rho0G) || !(T0 > 0.0) || !std::isfinite(T0)))
    return fail(RBOS_E_RANGE, "rho0G and T0 must be positive and finite");
  hipError_t e = rbos::launch_field_pack(nx, ny, nz, src, from_t, (float)rho0G, (float)T0, dtype, (float)scale,
                                         (float)offset, field, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(RBOS_E_HIP, "field pack launch failed: %s", hipGetErrorString(e));
  return RBOS_OK;
}

int rbos_field_from_temperature(int32_t nx, int32_t ny, int32_t nz, const float* T, double rho0G, double T0,
                                int32_t dtype, double enc_scale, double enc_offset, void* field, void* stream) {
  return field_common(nx, ny, nz, T, 1, rho0G, T0, dtype, enc_scale, enc_offset, field, stream);
}

int rbos_field_encode(int32_t nx, int32_t ny, int32_t nz, const float* delta, int32_t dtype, double enc_scale,
                      double enc_offset, void* field, void* stream) {
  return field_common(nx, ny, nz, delta, 0, 0.0, 0.0, dtype, enc_scale, enc_offset, field, stream);
}

// Largest power of two s with s * max |delta - c| <= 2^14 over delta in [lo, hi] (|delta - c|
// is convex, so its maximum is at an end of the range); 1 for FP32 or a zero range.
static double code_scale(int32_t dtype, double lo, double hi, double c) {
  if (!valid_dtype(dtype)) return 0.0;
  if (rbos::code_type(dtype) == rbos::DT_F32) return 1.0;
  if (!std::isfinite(lo) || !std::isfinite(hi) || !std::isfinite(c) || lo > hi) return 0.0;
  const double m = std::max(std::fabs(lo - c), std::fabs(hi - c));
  if (m == 0.0) return 1.0;
  int e = 0;
  const double f = std::frexp(m, &e);  // m = f 2^e, f in [0.5, 1)
  return std::ldexp(1.0, (f == 0.5 ? 15 : 14) - e);
}

double rbos_code_scale(int32_t dtype, double delta_lo, double delta_hi, double enc_offset) {
  return code_scale(dtype, delta_lo, delta_hi, enc_offset);
}

double rbos_code_scale_temperature(int32_t dtype, double T_lo, double T_hi, double rho0G, double T0,
                                   double enc_offset) {
  if (!(T_lo > 0.0) || !(T_hi >= T_lo) || !std::isfinite(T_hi) || !(rho0G > 0.0) || !std::isfinite(rho0G) ||
      !(T0 > 0.0) || !std::isfinite(T0))
    return 0.0;
  // eta - 1 = rho0 G T0 / T decreases with T
  return code_scale(dtype, rho0G * T0 / T_hi, rho0G * T0 / T_lo, enc_offset);
}

size_t rbos_ckpt_bytes(const rbos_scene* S) {
  if (!S || S->ckpt_stride <= 0 || S->max_steps < 1 || S->n_pixels < 0 || S->spp < 1) return 0;
  // a per-ray header, then checkpoint slots for steps k, 2k, ... below max_steps
  // (6 floats per ray and slot; none for the quasi-linear tracer)
  return (rbos::RAY_HEADER + (size_t)ckpt_slots(S) * 6) * (size_t)ckpt_entries(S) * sizeof(float);
}

size_t rbos_workspace_bytes(const rbos_scene* scenes, int32_t n_scenes) {
  if (!scenes || n_scenes < 0) return 0;
  Launch L;
  // tile counts differ with the tile shape only for full images; take the largest
  size_t best = 0;
  const int shapes[7][2] = {{1, 64}, {2, 32}, {4, 16}, {8, 8}, {16, 4}, {32, 2}, {64, 1}};
  for (auto& sh : shapes) {
    L.tile_w = sh[0];
    L.tile_h = sh[1];
    Layout y = layout(scenes, n_scenes, L);
    if (y.total > best) best = y.total;
  }
  return best;
}

int rbos_trace_forward(const rbos_scene* scenes, int32_t n_scenes, const rbos_trace_out* outs,
                       const rbos_launch* launch, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  Prepared P;
  int rc = prepare(scenes, n_scenes, launch, workspace, ws_bytes, false, P);
  if (rc) return rc;
  if (n_scenes > 0 && !outs) return fail(RBOS_E_NULL, "outs is NULL");
  for (int i = 0; i < n_scenes; ++i) {
    const rbos_trace_out& o = outs[i];
    const bool rays = scenes[i].n_pixels > 0;
    if (rays && (!o.wall_uv || !o.wall_duv || !o.n_steps || !o.status))
      return fail(RBOS_E_NULL, "scene %d: wall_uv, wall_duv, n_steps and status are required", i);
    if (rays && scenes[i].ckpt_stride > 0 && !o.ckpt)
      return fail(RBOS_E_NULL, "scene %d: ckpt_stride > 0 needs ckpt", i);
    SceneDev& d = P.table[i];
    d.uv = o.wall_uv;
    d.duv = o.wall_duv;
    d.n_steps = o.n_steps;
    d.status = o.status;
    d.ckpt = scenes[i].ckpt_stride > 0 ? o.ckpt : nullptr;
    d.wall_dir = o.wall_dir;
  }
  if (n_scenes == 0 || P.Y.total_tiles == 0) return RBOS_OK;
  rbos::LaunchPlan plan{};
  hipStream_t stream_h = static_cast<hipStream_t>(stream);
  rc = finish_launch(P, workspace, stream_h, plan);
  if (rc) return rc;
  hipError_t e = rbos::launch_trace_fwd(plan, stream_h);
  if (e != hipSuccess) return fail(RBOS_E_HIP, "forward launch failed: %s", hipGetErrorString(e));
  return RBOS_OK;
}

int rbos_render(const rbos_scene* scenes, int32_t n_scenes, const rbos_trace_out* outs, const rbos_render_io* io,
                void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  Prepared P;
  int rc = prepare(scenes, n_scenes, nullptr, workspace, ws_bytes, true, P);
  if (rc) return rc;
  if (n_scenes > 0 && (!outs || !io)) return fail(RBOS_E_NULL, "outs or io is NULL");
  for (int i = 0; i < n_scenes; ++i) {
    const bool rays = scenes[i].n_pixels > 0;
    const bool radio = scenes[i].radiometry != 0;
    if (rays && (!outs[i].wall_duv || !outs[i].status))
      return fail(RBOS_E_NULL, "scene %d: wall_duv and status are required", i);
    if (rays && radio && !outs[i].wall_dir)
      return fail(RBOS_E_NULL, "scene %d: radiometry needs the forward's wall_dir", i);
    if (rays && !io[i].image) return fail(RBOS_E_NULL, "scene %d: image is required", i);
    if ((io[i].dL_duv || io[i].loss || io[i].dL_ddir) && !io[i].target)
      return fail(RBOS_E_NULL, "scene %d: dL_duv, dL_ddir and loss need a target", i);
    if (rays && radio && io[i].dL_duv && !io[i].dL_ddir)
      return fail(RBOS_E_NULL, "scene %d: with radiometry, dL_duv needs dL_ddir as well", i);
    SceneDev& d = P.table[i];
    d.duv = outs[i].wall_duv;
    d.status = outs[i].status;
    d.wall_dir = outs[i].wall_dir;
    d.target = io[i].target;
    d.image = io[i].image;
    d.dL_duv = io[i].dL_duv;
    d.dL_ddir = radio ? io[i].dL_ddir : nullptr;
    d.loss = io[i].loss;
  }
  if (n_scenes == 0) return RBOS_OK;
  rbos::LaunchPlan plan{};
  hipStream_t stream_h = static_cast<hipStream_t>(stream);
  rc = finish_launch(P, workspace, stream_h, plan);
  if (rc) return rc;
  hipError_t e = rbos::launch_render(plan, stream_h);
  if (e != hipSuccess) return fail(RBOS_E_HIP, "render launch failed: %s", hipGetErrorString(e));
  return RBOS_OK;
}

int rbos_trace_adjoint(const rbos_scene* scenes, int32_t n_scenes, const rbos_trace_out* outs,
                       const rbos_adjoint_io* io, const rbos_launch* launch, void* workspace, size_t ws_bytes,
                       void* stream) {
  g_err.clear();
  Prepared P;
  int rc = prepare(scenes, n_scenes, launch, workspace, ws_bytes, false, P);
  if (rc) return rc;
  rc = adjoint_bind(P, scenes, n_scenes, outs, io);
  if (rc) return rc;
  return adjoint_enqueue(P, n_scenes, workspace, static_cast<hipStream_t>(stream));
}

int rbos_trace_adjoint_noalloc(const rbos_scene* scenes, int32_t n_scenes, const rbos_trace_out* outs,
                               const rbos_adjoint_io* io, const rbos_launch* launch, void* stream) {
  g_err.clear();
  Prepared P;
  // host validation against the scratch size first (no device call): the workspace
  // pointer given here is only checked for alignment and never dereferenced
  int rc = prepare(scenes, n_scenes, launch, reinterpret_cast<void*>(uintptr_t{256}), NOALLOC_SCRATCH_BYTES, false, P);
  if (rc == RBOS_E_WORKSPACE)
    return fail(RBOS_E_WORKSPACE,
                "rbos_trace_adjoint_noalloc: these scenes need %zu bytes of device scratch, the static buffer "
                "holds %zu (use rbos_trace_adjoint with a workspace)",
                P.Y.total, NOALLOC_SCRATCH_BYTES);
  if (rc) return rc;
  rc = adjoint_bind(P, scenes, n_scenes, outs, io);
  if (rc) return rc;
  if (n_scenes == 0 || P.Y.total_tiles == 0) return RBOS_OK;
  void* scratch_dev = nullptr;
  rc = noalloc_scratch(&scratch_dev);
  if (rc) return rc;
  return adjoint_enqueue(P, n_scenes, scratch_dev, static_cast<hipStream_t>(stream));
}

size_t rbos_mlp_param_count(int32_t width, int32_t depth) {
  if (width != rbos::MLP_WIDTH || depth < 1 || depth > rbos::MLP_MAX_DEPTH) return 0;
  const size_t w = (size_t)width;
  return 3 * w + w + (size_t)(depth - 1) * (w * w + w) + w * rbos::MLP_OUT + rbos::MLP_OUT;
}

size_t rbos_mlp_workspace_bytes(int32_t width, int32_t depth, int64_t n_points) {
  if (rbos_mlp_param_count(width, depth) == 0 || n_points < 0) return 0;
  return rbos::mlp_work_bytes(depth, n_points);
}

}  // extern "C"

namespace {

enum { MLP_WS_PLAIN = 0, MLP_WS_JET = 1 };

int mlp_prepare(const rbos_mlp* m, const float* points, int64_t n, const int32_t* grid, void* ws, size_t ws_bytes,
                int ws_kind, rbos::MlpDev& M, rbos::MlpWork& W) {
  if (!m) return fail(RBOS_E_NULL, "mlp is NULL");
  if (rbos_mlp_param_count(m->width, m->depth) == 0)
    return fail(RBOS_E_UNSUPPORTED, "mlp: width must be %d and depth in [1, %d] (got %d, %d)", rbos::MLP_WIDTH,
                rbos::MLP_MAX_DEPTH, m->width, m->depth);
  if (!m->params) return fail(RBOS_E_NULL, "mlp: params is NULL");
  if (!finite3(m->box_lo) || !finite3(m->box_hi) || !(m->box_lo[0] < m->box_hi[0]) ||
      !(m->box_lo[1] < m->box_hi[1]) || !(m->box_lo[2] < m->box_hi[2]))
    return fail(RBOS_E_RANGE, "mlp: box must be finite with lo < hi");
  if (n < 0 || n > (1LL << 31)) return fail(RBOS_E_SHAPE, "mlp: n_points must be in [0, 2^31]");
  std::memset(&M, 0, sizeof M);
  if (!points && n > 0) {
    if (!grid) return fail(RBOS_E_NULL, "mlp: points and grid_dims are both NULL");
    if (grid[0] < 1 || grid[1] < 1 || grid[2] < 1 || (long long)grid[0] * grid[1] * grid[2] != n)
      return fail(RBOS_E_SHAPE, "mlp: grid_dims must be positive with nx*ny*nz == n_points");
    M.nx = grid[0];
    M.ny = grid[1];
    M.nz = grid[2];
  }
  if (n > 0) {
    if (!ws) return fail(RBOS_E_WORKSPACE, "mlp: workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(RBOS_E_WORKSPACE, "mlp: workspace must be 256-byte aligned");
    const size_t need = ws_kind == MLP_WS_JET ? rbos::mlp_jet_work_bytes(m->depth, n) : rbos::mlp_work_bytes(m->depth, n);
    if (ws_bytes < need) return fail(RBOS_E_WORKSPACE, "mlp: workspace too small: %zu < %zu bytes", ws_bytes, need);
  }
  M.depth = m->depth;
  M.params = m->params;
  int off = 0;
  for (int l = 0; l <= m->depth; ++l) {
    const int fi = l == 0 ? 3 : rbos::MLP_WIDTH, fo = l == m->depth ? rbos::MLP_OUT : rbos::MLP_WIDTH;
    M.off_w[l] = off;
    off += fi * fo;
    M.off_b[l] = off;
    off += fo;
  }
  M.n = n;
  M.points = points;
  for (int a = 0; a < 3; ++a) {
    const double sc = 2.0 / (m->box_hi[a] - m->box_lo[a]);
    M.xs[a] = (float)sc;
    M.xo[a] = (float)(-m->box_lo[a] * sc - 1.0);
  }
  if (n > 0 && ws_kind == MLP_WS_PLAIN) rbos::mlp_work_carve(ws, m->depth, n, W);
  return RBOS_OK;
}

}  // namespace

extern "C" {

int rbos_mlp_forward(const rbos_mlp* mlp, const float* points, int64_t n_points, const int32_t* grid_dims,
                     float* out, float* T, double T0, double T_in, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  rbos::MlpDev M;
  rbos::MlpWork W;
  int rc = mlp_prepare(mlp, points, n_points, grid_dims, workspace, ws_bytes, MLP_WS_PLAIN, M, W);
  if (rc) return rc;
  if (T && !(std::isfinite(T0) && std::isfinite(T_in))) return fail(RBOS_E_RANGE, "mlp: T0 and T_in must be finite");
  if (n_points == 0) return RBOS_OK;
  hipError_t e = rbos::launch_mlp_forward(M, W, out, T, (float)T0, (float)(T_in - T0), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(RBOS_E_HIP, "mlp forward launch failed: %s", hipGetErrorString(e));
  return RBOS_OK;
}

int rbos_mlp_backward(const rbos_mlp* mlp, const float* points, int64_t n_points, const int32_t* grid_dims,
                      const float* dL_dout, float* dparams, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  rbos::MlpDev M;
  rbos::MlpWork W;
  int rc = mlp_prepare(mlp, points, n_points, grid_dims, workspace, ws_bytes, MLP_WS_PLAIN, M, W);
  if (rc) return rc;
  if (!dparams) return fail(RBOS_E_NULL, "mlp: dparams is NULL");
  if (n_points > 0 && !dL_dout) return fail(RBOS_E_NULL, "mlp: dL_dout is NULL");
  if (n_points == 0) return RBOS_OK;
  hipError_t e = rbos::launch_mlp_backward(M, W, dL_dout, dparams, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(RBOS_E_HIP, "mlp backward launch failed: %s", hipGetErrorString(e));
  return RBOS_OK;
}

int rbos_mlp_bos_seed(int64_t n, const float* T, const double* grad_delta, double rho0G, double T0, double T_in,
                      float* dL_dout, void* stream) {
  g_err.clear();
  if (n < 0) return fail(RBOS_E_SHAPE, "n < 0");
  if (n > 0 && (!T || !grad_delta || !dL_dout)) return fail(RBOS_E_NULL, "T, grad_delta and dL_dout are required");
  if (!(rho0G > 0.0) || !std::isfinite(rho0G) || !(T0 > 0.0) || !std::isfinite(T0) || !std::isfinite(T_in))
    return fail(RBOS_E_RANGE, "rho0G and T0 must be positive and finite, T_in finite");
  hipError_t e = rbos::launch_mlp_bos_seed(n, T, grad_delta, rho0G, T0, T_in - T0, dL_dout,
                                           static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(RBOS_E_HIP, "seed launch failed: %s", hipGetErrorString(e));
  return RBOS_OK;
}

size_t rbos_mlp_fit_workspace_bytes(int64_t n_points) {
  if (n_points < 0) return 0;
  return ((size_t)((n_points + 255) / 256) * sizeof(float) + 255) / 256 * 256 + 256;
}

int rbos_mlp_fit_seed(int64_t n, const float* out, const float* target, const double* norms, float* dL_dout,
                      float* loss, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (n < 0 || n > (1LL << 31)) return fail(RBOS_E_SHAPE, "n must be in [0, 2^31]");
  if (!norms) return fail(RBOS_E_NULL, "norms is NULL");
  for (int k = 0; k < rbos::MLP_OUT; ++k)
    if (!(norms[k] > 0.0) || !std::isfinite(norms[k])) return fail(RBOS_E_RANGE, "norms must be positive and finite");
  if (n > 0 && (!out || !target || !dL_dout)) return fail(RBOS_E_NULL, "out, target and dL_dout are required");
  if (loss) {
    if (!workspace) return fail(RBOS_E_WORKSPACE, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(RBOS_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < rbos_mlp_fit_workspace_bytes(n)) return fail(RBOS_E_WORKSPACE, "workspace too small");
  }
  hipError_t e = rbos::launch_mlp_fit_seed(n, out, target, norms, dL_dout, loss, static_cast<float*>(workspace),
                                           static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(RBOS_E_HIP, "fit seed launch failed: %s", hipGetErrorString(e));
  return RBOS_OK;
}

size_t rbos_mlp_pde_workspace_bytes(int32_t width, int32_t depth, int64_t n_points) {
  if (rbos_mlp_param_count(width, depth) == 0 || n_points < 0) return 0;
  return rbos::mlp_jet_work_bytes(depth, n_points);
}

int rbos_mlp_pde_loss(const rbos_mlp* mlp, const rbos_pde* pde, const float* points, int64_t n_points, float* loss,
                      float* dparams, float* residuals, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!pde) return fail(RBOS_E_NULL, "pde is NULL");
  if (n_points > 0 && !points) return fail(RBOS_E_NULL, "points is NULL");
  if (n_points > (1LL << 28)) return fail(RBOS_E_SHAPE, "n_points must be <= 2^28");
  rbos::MlpDev M;
  rbos::MlpWork W;
  int rc = mlp_prepare(mlp, points, n_points, nullptr, workspace, ws_bytes, MLP_WS_JET, M, W);
  if (rc) return rc;
  if (!(pde->Re > 0.0) || !(pde->Pe > 0.0) || !(pde->L > 0.0) || !std::isfinite(pde->Re) || !std::isfinite(pde->Pe) ||
      !std::isfinite(pde->Ri) || !std::isfinite(pde->L))
    return fail(RBOS_E_RANGE, "pde: Re, Pe, L must be positive and finite, Ri finite");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(pde->gamma[k]) || pde->gamma[k] < 0.0) return fail(RBOS_E_RANGE, "pde: gamma must be >= 0");
  rbos::PdeConst P;
  for (int a = 0; a < 3; ++a) P.s[a] = (float)(2.0 * pde->L / (mlp->box_hi[a] - mlp->box_lo[a]));
  P.inv_re = (float)(1.0 / pde->Re);
  P.inv_pe = (float)(1.0 / pde->Pe);
  P.ri = (float)pde->Ri;
  for (int k = 0; k < 3; ++k) P.g[k] = (float)pde->gamma[k];
  hipError_t e = rbos::launch_mlp_pde(M, workspace, P, loss, dparams, residuals, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(RBOS_E_HIP, "pde launch failed: %s", hipGetErrorString(e));
  return RBOS_OK;
}

size_t rbos_struct_layout(int32_t which, size_t* offsets, int32_t max_fields) {
#define OFF(T, f) offsetof(T, f)
  std::vector<size_t> o;
  size_t sz = 0;
  switch (which) {
    case 0:
      o = {OFF(rbos_scene, nx), OFF(rbos_scene, ny), OFF(rbos_scene, nz), OFF(rbos_scene, box_lo),
           OFF(rbos_scene, box_hi), OFF(rbos_scene, dtype), OFF(rbos_scene, enc_scale), OFF(rbos_scene, enc_offset),
           OFF(rbos_scene, field), OFF(rbos_scene, cam_pos), OFF(rbos_scene, cam_fwd), OFF(rbos_scene, cam_right),
           OFF(rbos_scene, cam_up), OFF(rbos_scene, cam_fov_x_deg), OFF(rbos_scene, width), OFF(rbos_scene, height),
           OFF(rbos_scene, pixel_ids), OFF(rbos_scene, n_pixels), OFF(rbos_scene, wall_origin),
           OFF(rbos_scene, wall_normal), OFF(rbos_scene, wall_u), OFF(rbos_scene, wall_v), OFF(rbos_scene, wall_mode),
           OFF(rbos_scene, pattern), OFF(rbos_scene, pat_w), OFF(rbos_scene, pat_h), OFF(rbos_scene, pat_extent_u),
           OFF(rbos_scene, pat_extent_v), OFF(rbos_scene, proj_pos), OFF(rbos_scene, proj_fwd),
           OFF(rbos_scene, proj_right), OFF(rbos_scene, proj_up), OFF(rbos_scene, proj_fov_x_deg),
           OFF(rbos_scene, step), OFF(rbos_scene, max_steps), OFF(rbos_scene, ckpt_stride), OFF(rbos_scene, tracer),
           OFF(rbos_scene, spp), OFF(rbos_scene, seed), OFF(rbos_scene, radiometry)};
      sz = sizeof(rbos_scene);
      break;
    case 1:
      o = {OFF(rbos_trace_out, wall_uv), OFF(rbos_trace_out, wall_duv), OFF(rbos_trace_out, n_steps),
           OFF(rbos_trace_out, status), OFF(rbos_trace_out, ckpt), OFF(rbos_trace_out, wall_dir)};
      sz = sizeof(rbos_trace_out);
      break;
    case 2:
      o = {OFF(rbos_render_io, target), OFF(rbos_render_io, image), OFF(rbos_render_io, dL_duv),
           OFF(rbos_render_io, loss), OFF(rbos_render_io, dL_ddir)};
      sz = sizeof(rbos_render_io);
      break;
    case 3:
      o = {OFF(rbos_adjoint_io, dL_duv), OFF(rbos_adjoint_io, grad), OFF(rbos_adjoint_io, dL_ddir)};
      sz = sizeof(rbos_adjoint_io);
      break;
    case 4:
      o = {OFF(rbos_launch, tile_w), OFF(rbos_launch, tile_h), OFF(rbos_launch, waves_per_block),
           OFF(rbos_launch, persistent), OFF(rbos_launch, blocks_per_cu)};
      sz = sizeof(rbos_launch);
      break;
    case 5:
      o = {OFF(rbos_mlp, width), OFF(rbos_mlp, depth), OFF(rbos_mlp, params), OFF(rbos_mlp, box_lo),
           OFF(rbos_mlp, box_hi)};
      sz = sizeof(rbos_mlp);
      break;
    case 6:
      o = {OFF(rbos_pde, Re), OFF(rbos_pde, Pe), OFF(rbos_pde, Ri), OFF(rbos_pde, L), OFF(rbos_pde, gamma)};
      sz = sizeof(rbos_pde);
      break;
    default:
      return 0;
  }
#undef OFF
  if (offsets)
    for (int i = 0; i < (int)o.size() && i < max_fields; ++i) offsets[i] = o[i];
  return sz;
}

}  // extern "C"
