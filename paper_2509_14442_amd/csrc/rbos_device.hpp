// rbos_device.hpp -- device-side building blocks shared by the librbos kernels.
//
//  * double-float arithmetic (pairs of binary32 values; Knuth two-sum, Dekker fast
//    two-sum, FMA two-product) for the per-ray geometry that needs ~1e-9 m accuracy:
//    camera ray, box entry, straight-line base of the ray, wall and projector maps;
//  * the device scene record built by the host from an rbos_scene;
//  * the cell-record field layout (with a one-voxel apron that repeats the edge voxels,
//    so clamp-to-edge needs no per-axis branching) and the trilinear sampler (value,
//    gradient, mixed second derivatives) of the cell-centred grid;
//  * one step of Sharma's Runge-Kutta-Nystrom scheme for Eq. (1) in grid units.
//
// Everything here is compiled with -ffp-contract=off: fused multiply-adds appear only
// where written (fmaf), so the forward kernel and the adjoint's replay of it perform
// bit-identical arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbos {

// ------------------------------------------------------------------------------------
// global-memory access through pointers read from the scene record: the compiler cannot
// tell that they address global memory and would emit flat instructions, which also
// count in the LDS wait counter (so every LDS wait would wait for the field gathers).
// ------------------------------------------------------------------------------------
#define RBOS_GLOBAL __attribute__((address_space(1)))
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const RBOS_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(RBOS_GLOBAL T*)p = v;
}
// Streaming store (non-temporal hint): data written once and read back much later, such
// as the checkpoints, then does not displace the field records from the caches.
template <class T>
__device__ __forceinline__ void gst_stream(T* p, T v) {
  __builtin_nontemporal_store(v, (RBOS_GLOBAL T*)p);
}
__device__ __forceinline__ void gatomic_add(double* p, double v) {
  __builtin_amdgcn_global_atomic_fadd_f64((RBOS_GLOBAL double*)p, v);
}

// ------------------------------------------------------------------------------------
// double-float
// ------------------------------------------------------------------------------------
struct df {
  float hi, lo;
};

__device__ __forceinline__ df dd_two_sum(float a, float b) {
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
// requires |a| >= |b| (or a == 0)
__device__ __forceinline__ df dd_fast(float a, float b) {
  float s = a + b;
  float e = b - (s - a);
  return {s, e};
}
__device__ __forceinline__ df dd_add(df a, df b) {
  df s = dd_two_sum(a.hi, b.hi);
  df t = dd_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_fast(s.hi, s.lo);
  s.lo += t.lo;
  return dd_fast(s.hi, s.lo);
}
__device__ __forceinline__ df dd_neg(df a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ df dd_sub(df a, df b) { return dd_add(a, dd_neg(b)); }
__device__ __forceinline__ df dd_add_f(df a, float b) {
  df s = dd_two_sum(a.hi, b);
  s.lo += a.lo;
  return dd_fast(s.hi, s.lo);
}
__device__ __forceinline__ df dd_mul(df a, df b) {
  float p = a.hi * b.hi;
  float e = fmaf(a.hi, b.hi, -p);
  e = fmaf(a.hi, b.lo, e);
  e = fmaf(a.lo, b.hi, e);
  return dd_fast(p, e);
}
__device__ __forceinline__ df dd_mul_f(df a, float b) {
  float p = a.hi * b;
  float e = fmaf(a.hi, b, -p);
  e = fmaf(a.lo, b, e);
  return dd_fast(p, e);
}
__device__ __forceinline__ df dd_div(df a, df b) {
  float q1 = a.hi / b.hi;
  df r = dd_sub(a, dd_mul_f(b, q1));
  float q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul_f(b, q2));
  float q3 = r.hi / b.hi;
  return dd_add_f(dd_fast(q1, q2), q3);
}
__device__ __forceinline__ df dd_sqrt(df a) {
  if (!(a.hi > 0.0f)) return {0.0f, 0.0f};
  float s = sqrtf(a.hi);
  float p = s * s;
  float pe = fmaf(s, s, -p);
  float e = (((a.hi - p) - pe) + a.lo) / (2.0f * s);
  return dd_fast(s, e);
}
__device__ __forceinline__ bool dd_lt(df a, df b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ __forceinline__ df dd_dot3(const df* a, const df* b) {
  return dd_add(dd_add(dd_mul(a[0], b[0]), dd_mul(a[1], b[1])), dd_mul(a[2], b[2]));
}
__device__ __forceinline__ float dd_to_f(df a) { return a.hi + a.lo; }

// ------------------------------------------------------------------------------------
// device scene record (host-built; see abi.hip)
// ------------------------------------------------------------------------------------
struct SceneDev {
  // field
  int n[3];            // voxels per axis
  int P0, P01;         // record strides: cell records (nx+1), (nx+1)(ny+1); x-pairs (nx+1), (nx+1)(ny+2)
  int P1;              // P01 / P0
  int dtype;
  const void* field;   // cell records, starting with cell (-1, -1, -1); cells -1 .. n-1 on every axis
  float dec;           // 1 / enc_scale
  float inv_dec;       // enc_scale
  float one_plus_off;  // 1 + enc_offset (binary32)
  float off;           // enc_offset (binary32)
  float km[3];         // dec / voxel^2: force factor in grid units
  float vox[3];        // voxel size (m)
  float lo_f[3];       // box lo (m)
  float hi_bound[3];   // n + 1/2: box faces in grid units are 1/2 and n + 1/2
  float n_f[3];        // n (binary32)
  unsigned rec_div_m[2];  // record index r (< 2^27) / P0 and / P01 as (r * m) >> s
  int rec_div_s[2];
  df lo[3];            // box lo (m)
  df hi[3];            // box hi (m)
  df inv_vox[3];       // 1 / voxel size
  // integrator
  df h;                // step in t
  float hf, h_2, h_6, h2_8, h2_2, h2_6;
  // stage coefficients of the force in code units (eta dq/du_a), per axis:
  // h^2/8 km_a (P2), h^2/2 km_a (P3), h^2/6 km_a (position), h/6 km_a (velocity)
  float c_p2[3], c_p3[3], c_x[3], c_v[3];
  float c_x2[3], c_v4[3];  // 2 c_x, 4 c_v: the second stage's weights in the adjoint
  double inv_dec_d;        // 1 / dec (binary64): scales the adjoint's monomial totals
  int max_steps, ckpt_k, ckpt_slots;
  int tracer;          // 0 nonlinear, 1 quasi-linear (forces on the entry line)
  long long ckpt_pad;  // entries per checkpoint component (a multiple of 64)
  int ckpt_tx;         // full image: 8 x 8 pixel blocks per image row
  // camera
  df cam_pos[3], cam_fwd[3], cam_right[3], cam_up[3];
  df cam_ax;           // tan(fov_x / 2) / width
  df cam_cx;           // tan(fov_x / 2)
  df cam_cy;           // tan(fov_x / 2) * height / width
  int width, height;
  const int* pixel_ids;
  int n_pix;           // pixels traced (length of pixel_ids, or width * height)
  int n_rays;          // n_pix * spp
  int spp;             // rays per pixel (Eq. 2); ray r = s * n_pix + i
  unsigned int seed;   // sub-pixel sample key
  int radiometry;      // weight radiance by |<n_w, v_w>| / |X_w - c|
  int tile_w, tile_h, tiles_x, n_tiles, tile_begin;
  int tiles_plane;     // tiles per sample plane
  long long ckpt_plane;  // checkpoint entries per sample plane
  // wall
  df wall_org[3], wall_n[3], wall_u[3], wall_v[3];
  float wall_n_f[3], wall_u_f[3], wall_v_f[3], wall_org_f[3];
  int wall_mode;
  const float* pattern;
  int pat_w, pat_h;
  df pat_half_u, pat_half_v;  // printed: extent / 2
  df pat_inv_tu, pat_inv_tv;  // printed: texels per metre
  df proj_pos[3], proj_fwd[3], proj_right[3], proj_up[3];
  df proj_inv_tx, proj_inv_ty;  // 1 / tan(fov_x/2), 1 / (tan(fov_x/2) * pat_h / pat_w)
  // forward outputs
  float* uv;
  float* duv;
  int* n_steps;
  unsigned char* status;
  float* ckpt;
  float* wall_dir;
  // render io
  const float* target;
  float* image;
  float* dL_duv;
  float* dL_ddir;
  float* loss;
  int render_block_begin, render_blocks;
  // adjoint io
  const float* adj_dL_duv;
  const float* adj_dL_ddir;
  double* grad;
};

enum : int {
  RAY_MISSED_BOX = 1,
  RAY_TRUNCATED = 2,
  RAY_NO_WALL_HIT = 4,
  RAY_NONFINITE = 8,
  RAY_OFF_PATTERN = 16
};

// Storage formats: the code type (FP32, FP16, BF16) of eta - 1, stored as cell records
// (0, 1, 2) or as x-pairs (3, 4, 5; see fetch_cell).
enum : int { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2, DT_F32_XPAIR = 3, DT_F16_XPAIR = 4, DT_BF16_XPAIR = 5 };

__host__ __device__ constexpr int code_type(int dt) { return dt % 3; }
__host__ __device__ constexpr bool is_xpair(int dt) { return dt >= 3; }

// ------------------------------------------------------------------------------------
// work decomposition: XCD-aware block order, tiles of 64 rays
// ------------------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so that each XCD
// works on runs of XCD_RUN consecutive blocks (neighbouring rays share field cells, and
// each XCD has its own L2), taking every 8th run. Contiguous eighths of the image would
// give the XCDs unequal work: rays that leave the box through its top or bottom face
// are short, and the XCDs holding those rows fell idle early (forward 1.86 -> 1.75 ms
// on the 1M-ray room with runs of 8 blocks). Blocks past the last whole round of runs
// keep their own index.
constexpr int XCD_RUN = 8;

__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
  const int full = nblocks / (8 * XCD_RUN);
  if (b >= full * 8 * XCD_RUN) return b;
  const int x = b & 7, k = b >> 3;
  return ((k / XCD_RUN) * 8 + x) * XCD_RUN + k % XCD_RUN;
}

// The persistent kernels' per-XCD queues (in the adjoint, positions in its tile order):
// XCD x owns runs of TILE_RUN tiles, every 8th run (so each XCD gets rows from the whole
// image and an even share of the work), then an eighth of the tiles past the last whole
// round of runs.
constexpr int TILE_RUN = 32;

__device__ __forceinline__ void xcd_tile_range(int total, int x, int& b, int& e) {
  const int full = total / (8 * TILE_RUN);
  const int rem = total - full * 8 * TILE_RUN;
  b = x * full * TILE_RUN + (int)(((long long)rem * x) >> 3);
  e = (x + 1) * full * TILE_RUN + (int)(((long long)rem * (x + 1)) >> 3);
}

// i-th tile owned by XCD x (0 <= i < the size of its range)
__device__ __forceinline__ int xcd_tile(int total, int x, int i) {
  const int full = total / (8 * TILE_RUN);
  if (i < full * TILE_RUN) return ((i / TILE_RUN) * 8 + x) * TILE_RUN + i % TILE_RUN;
  const int rem = total - full * 8 * TILE_RUN;
  return full * 8 * TILE_RUN + (int)(((long long)rem * x) >> 3) + (i - full * TILE_RUN);
}

// The same value in every lane, made visible as such to the compiler (kept in an SGPR, so
// that the scene record it indexes is read with scalar loads).
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// scene owning global tile index t (scenes are sorted by tile_begin)
__device__ __forceinline__ int find_scene(const SceneDev* scenes, int n_scenes, int t) {
  int lo = 0, hi = n_scenes - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (scenes[mid].tile_begin <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Entry of ray r (pixel pix, sample s) in every checkpoint component: per sample plane,
// the image in 8 x 8 pixel blocks, row-major over blocks and within a block, so the 64
// rays of an 8 x 8 tile read and write one contiguous 256-byte run; with a pixel-id
// list, r itself.
__device__ __forceinline__ int ckpt_entry(const SceneDev& S, int r, int pix, int s) {
  if (S.pixel_ids) return r;
  const int row = pix / S.width, col = pix - row * S.width;
  return (int)(s * S.ckpt_plane) + (((row >> 3) * S.ckpt_tx + (col >> 3)) << 6) + ((row & 7) << 3) + (col & 7);
}

// Ray index r, pixel and sample of lane `lane` in scene tile `tile`; false if none. Tiles
// are grouped by sample plane (every tile holds one sample of 64 neighbouring pixels),
// so `s` is the same in every lane.
__device__ __forceinline__ bool tile_ray(const SceneDev& S, int tile, int lane, int& r, int& pix, int& s) {
  s = tile / S.tiles_plane;
  const int t = tile - s * S.tiles_plane;
  if (S.pixel_ids) {
    const int i = t * 64 + lane;
    if (i >= S.n_pix) return false;
    pix = gld(S.pixel_ids + i);
    r = s * S.n_pix + i;
    return true;
  }
  int tx = t % S.tiles_x, ty = t / S.tiles_x;
  int col = tx * S.tile_w + lane % S.tile_w;
  int row = ty * S.tile_h + lane / S.tile_w;
  if (col >= S.width || row >= S.height) return false;
  pix = row * S.width + col;
  r = s * S.n_pix + pix;
  return true;
}

// ------------------------------------------------------------------------------------
// per-ray geometry (double-float)
// ------------------------------------------------------------------------------------
struct Ray {
  df dir[3];     // unit camera ray direction
  bool entered;  // meets the field box
  df U0[3];      // box entry point in grid units, u = (x - lo)/voxel + 1/2
  bool wall0;    // the undeflected camera ray hits the wall
  df uv0[2];     // its wall coordinates
};

// Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) of the counter (c0, c1, 0, 0)
// under the key (k0, 0); returns the first two output words. Each round multiplies the
// even words by the two round constants, mixes the high halves with the odd words and
// the key, and the key steps by the Weyl increments.
__device__ __forceinline__ void philox2(unsigned int c0, unsigned int c1, unsigned int k0, unsigned int& x0,
                                        unsigned int& x1) {
  unsigned int c2 = 0u, c3 = 0u, k1 = 0u;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const unsigned int lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const unsigned int lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  x0 = c0;
  x1 = c1;
}

// Inverse CDF of the triangular density 1 - |x| on [-1, 1] at a 24-bit uniform u. u, 2u
// and 2 - 2u are exact in binary32; the one rounding of the square root moves the sample
// by under 1e-7 pixel.
__device__ __forceinline__ float tent_offset(unsigned int x) {
  const float u = (float)(x >> 8) * 0x1p-24f;
  return u < 0.5f ? sqrtf(2.0f * u) - 1.0f : 1.0f - sqrtf(2.0f - 2.0f * u);
}

// Image-plane coordinates 2 (col + 1/2 + ox) and 2 (row + 1/2 + oy) of sample s of pixel
// pix, summed exactly in double-float. Kept out of line: it runs once per ray, and inlined
// into the tracing kernels its temporaries raised their register allocation.
struct df2 {
  df x, y;
};
__device__ __attribute__((noinline)) df2 sample_point(int col, int row, unsigned int pix, unsigned int s,
                                                     unsigned int seed) {
  unsigned int x0, x1;
  philox2(pix, s, seed, x0, x1);
  return df2{dd_add_f(df{(float)(2 * col + 1), 0.0f}, 2.0f * tent_offset(x0)),
             dd_add_f(df{(float)(2 * row + 1), 0.0f}, 2.0f * tent_offset(x1))};
}

// Camera ray of sample s of pixel pix: through the pixel centre with one sample per pixel,
// else through the centre plus the sample's offset drawn from the triangular filter.
__device__ __forceinline__ void camera_ray(const SceneDev& S, int pix, int s, df dir[3]) {
  int col = pix % S.width, row = pix / S.width;
  df px, py;
  if (S.spp == 1) {
    px = dd_sub(dd_mul_f(S.cam_ax, (float)(2 * col + 1)), S.cam_cx);
    py = dd_sub(S.cam_cy, dd_mul_f(S.cam_ax, (float)(2 * row + 1)));
  } else {
    const df2 q = sample_point(col, row, (unsigned int)pix, (unsigned int)s, S.seed);
    px = dd_sub(dd_mul(S.cam_ax, q.x), S.cam_cx);
    py = dd_sub(S.cam_cy, dd_mul(S.cam_ax, q.y));
  }
  for (int a = 0; a < 3; ++a)
    dir[a] = dd_add(S.cam_fwd[a], dd_add(dd_mul(px, S.cam_right[a]), dd_mul(py, S.cam_up[a])));
  df len = dd_sqrt(dd_dot3(dir, dir));
  for (int a = 0; a < 3; ++a) dir[a] = dd_div(dir[a], len);
}

// slab test against the field box; t_in >= 0
__device__ __forceinline__ bool box_entry(const SceneDev& S, const df dir[3], df& t_in) {
  bool have_n = false;
  df tn = {0.0f, 0.0f}, tf = {0.0f, 0.0f};
  bool have_f = false;
  for (int a = 0; a < 3; ++a) {
    if (dir[a].hi != 0.0f) {
      df t1 = dd_div(dd_sub(S.lo[a], S.cam_pos[a]), dir[a]);
      df t2 = dd_div(dd_sub(S.hi[a], S.cam_pos[a]), dir[a]);
      df tmin = dd_lt(t1, t2) ? t1 : t2, tmax = dd_lt(t1, t2) ? t2 : t1;
      if (!have_n || dd_lt(tn, tmin)) tn = tmin;
      if (!have_f || dd_lt(tmax, tf)) tf = tmax;
      have_n = have_f = true;
    } else if (dd_lt(S.cam_pos[a], S.lo[a]) || dd_lt(S.hi[a], S.cam_pos[a])) {
      return false;
    }
  }
  df start = (have_n && tn.hi > 0.0f) ? tn : df{0.0f, 0.0f};
  if (!have_f) return false;  // degenerate direction
  if (!dd_lt(start, tf)) return false;
  t_in = start;
  return true;
}

// undeflected wall hit of the camera ray: (u0, v0)
__device__ __forceinline__ bool wall_hit_straight(const SceneDev& S, const df dir[3], df uv[2]) {
  df dn = dd_dot3(dir, S.wall_n);
  if (!(dn.hi < 0.0f)) return false;
  df w[3];
  for (int a = 0; a < 3; ++a) w[a] = dd_sub(S.wall_org[a], S.cam_pos[a]);
  df t = dd_div(dd_dot3(w, S.wall_n), dn);
  df r[3];
  for (int a = 0; a < 3; ++a) r[a] = dd_sub(dd_add(S.cam_pos[a], dd_mul(t, dir[a])), S.wall_org[a]);
  uv[0] = dd_dot3(r, S.wall_u);
  uv[1] = dd_dot3(r, S.wall_v);
  return true;
}

// ------------------------------------------------------------------------------------
// field: cell records or x-pairs, and the trilinear sampler
// ------------------------------------------------------------------------------------
// Cell records: the record of cell (i, j, k), i in [-1, n-1] per axis, is built from the 8
// corner codes q[a + 2b + 4c] = code(clamp(i+a), clamp(j+b), clamp(k+c)), indices clamped
// to the grid. FP16/BF16: the 8 codes, 16 bits each (16 B), two per 32-bit word. FP32: the
// 8 coefficients of the cell's trilinear polynomial in its fractions (u, v, w) (32 B, see
// corner_coefficients), so that value and derivatives need no differences. One sample is
// one 32-byte (two 16-byte loads) or 16-byte load at the record index
// rec = p0 + P0 p1 + P01 p2 of the padded cell (p = i + 1).
// X-pairs: entry (p0, r1, r2), p0 in [0, nx], r1 in [0, ny + 1], r2 in [0, nz + 1], holds
// the codes of voxels (clamp(p0 - 1), y, z) and (clamp(p0), y, z) with y = clamp(r1 - 1),
// z = clamp(r2 - 1): one FP32 pair (8 B) or two 16-bit codes in a 32-bit word. The cell
// p = (p0, p1, p2) reads the four entries rec, rec + P0, rec + P01, rec + P0 + P01 with
// rec = p0 + P0 p1 + P01 p2: four loads of 8 or 4 bytes instead of one record, over an
// array 4 (16-bit) to 8 (FP32) times smaller than the cell records.
// The 8 stored values of cell `rec`: the FP32 record's coefficients, else the corner codes.
template <int DT>
__device__ __forceinline__ void fetch_corners(const SceneDev& S, unsigned int rec, float c[8]) {
  // 32-bit byte offsets from the array start (at most 449^3 records of 32 B < 4 GiB), so
  // the load takes the array base from SGPRs and the offset from one VGPR
  const unsigned char* base = static_cast<const unsigned char*>(S.field);
  if constexpr (DT == DT_F32) {
    const f32x4* p = reinterpret_cast<const f32x4*>(base + (rec << 5));
    const f32x4 a = gld(p), b = gld(p + 1);
    c[0] = a.x; c[1] = a.y; c[2] = a.z; c[3] = a.w;
    c[4] = b.x; c[5] = b.y; c[6] = b.z; c[7] = b.w;
  } else if constexpr (DT == DT_F32_XPAIR) {
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const unsigned P0 = (unsigned)S.P0, P01 = (unsigned)S.P01;
    const f32x2 a = gld(reinterpret_cast<const f32x2*>(base + (rec << 3)));
    const f32x2 b = gld(reinterpret_cast<const f32x2*>(base + ((rec + P0) << 3)));
    const f32x2 d = gld(reinterpret_cast<const f32x2*>(base + ((rec + P01) << 3)));
    const f32x2 e = gld(reinterpret_cast<const f32x2*>(base + ((rec + P0 + P01) << 3)));
    c[0] = a.x; c[1] = a.y; c[2] = b.x; c[3] = b.y;
    c[4] = d.x; c[5] = d.y; c[6] = e.x; c[7] = e.y;
  } else {
    unsigned int v[4];
    if constexpr (is_xpair(DT)) {
      const unsigned P0 = (unsigned)S.P0, P01 = (unsigned)S.P01;
      v[0] = gld(reinterpret_cast<const unsigned int*>(base + (rec << 2)));
      v[1] = gld(reinterpret_cast<const unsigned int*>(base + ((rec + P0) << 2)));
      v[2] = gld(reinterpret_cast<const unsigned int*>(base + ((rec + P01) << 2)));
      v[3] = gld(reinterpret_cast<const unsigned int*>(base + ((rec + P0 + P01) << 2)));
    } else {
      const u32x4 w = gld(reinterpret_cast<const u32x4*>(base + (rec << 4)));
      v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (code_type(DT) == DT_F16) {
        // Plain v_cvt_f32_f16 on separated halves: left free, the compiler folds the
        // conversions into v_fma_mix_f32 / SDWA forms, which made the FP16 kernels ~10%
        // slower on gfx950. The empty asm statements only hide the values from that fold.
        unsigned lo16 = v[k] & 0xffffu, hi16 = v[k] >> 16;
        asm("" : "+v"(lo16), "+v"(hi16));
        c[2 * k] = (float)__builtin_bit_cast(_Float16, (unsigned short)lo16);
        c[2 * k + 1] = (float)__builtin_bit_cast(_Float16, (unsigned short)hi16);
        asm("" : "+v"(c[2 * k]), "+v"(c[2 * k + 1]));
      } else {
        c[2 * k] = __uint_as_float(v[k] << 16);
        c[2 * k + 1] = __uint_as_float(v[k] & 0xffff0000u);
      }
    }
  }
}

// Coefficients of the trilinear polynomial of a cell from its corner values q (index
// a + 2b + 4c): q(u, v, w) = sum_m C[m] u^(m & 1) v^(m >> 1 & 1) w^(m >> 2), i.e.
//   C0 = q0, C1 = q1 - q0, C2 = q2 - q0, C4 = q4 - q0,
//   C3 = (q3 - q2) - C1, C5 = (q5 - q4) - C1, C6 = (q6 - q4) - C2,
//   C7 = ((q7 - q6) - (q5 - q4)) - C3.
// The field encoder writes FP32 records this way (same operations, same order).
__host__ __device__ __forceinline__ void corner_coefficients(const float q[8], float C[8]) {
  const float d1 = q[1] - q[0], d3 = q[3] - q[2], d5 = q[5] - q[4], d7 = q[7] - q[6];
  C[0] = q[0];
  C[1] = d1;
  C[2] = q[2] - q[0];
  C[4] = q[4] - q[0];
  C[3] = d3 - d1;
  C[5] = d5 - d1;
  C[6] = (q[6] - q[4]) - C[2];
  C[7] = (d7 - d5) - C[3];
}

// The trilinear coefficients C[8] of cell `rec` (see corner_coefficients).
template <int DT>
__device__ __forceinline__ void fetch_cell(const SceneDev& S, unsigned int rec, float C[8]) {
  float c[8];
  fetch_corners<DT>(S, rec, c);
  if constexpr (DT == DT_F32) {
#pragma unroll
    for (int k = 0; k < 8; ++k) C[k] = c[k];  // FP32 records hold the coefficients
  } else {
    corner_coefficients(c, C);
  }
}

// Locate one axis: the point is u = bhi + small grid units (grid units count from one
// cell below the first voxel centre: u = (x - lo) / voxel + 1/2), with bhi exact. The
// padded cell index is p = floor(u) (cell i = p - 1 between centres i and i + 1) and
// f = u - p, computed without rounding u itself: bhi - floor(bhi) is exact, so f carries
// one rounding (~3e-8 voxel). p is clamped to [0, n]: the apron cells 0 and n repeat
// the edge voxels, so there the field is constant along the axis (edge value, zero
// derivative) for any f -- clamp-to-edge with half-open cells.
__device__ __forceinline__ void locate(float bhi, float small, float n_f, int& p, float& f) {
  const float fl = floorf(bhi);
  const float ff = (bhi - fl) + small;
  const float t = floorf(ff);
  f = ff - t;
  // integers far below 2^24 (or a non-finite position, mapped into [0, n])
  p = (int)__builtin_amdgcn_fmed3f(fl + t, 0.0f, n_f);
}

// As locate, plus the unclamped floor pu of u (NaN when the position is not finite).
__device__ __forceinline__ void locate_floor(float bhi, float small, float n_f, int& p, float& f, float& pu) {
  const float fl = floorf(bhi);
  const float ff = (bhi - fl) + small;
  const float t = floorf(ff);
  f = ff - t;
  pu = fl + t;
  p = (int)__builtin_amdgcn_fmed3f(pu, 0.0f, n_f);
}

struct Cell {
  int p[3];    // padded cell index i + 1 per axis, 0 .. n
  float f[3];  // fraction within the cell
};

__device__ __forceinline__ void locate3(const SceneDev& S, const float bhi[3], const float small[3], Cell& C) {
  locate(bhi[0], small[0], S.n_f[0], C.p[0], C.f[0]);
  locate(bhi[1], small[1], S.n_f[1], C.p[1], C.f[1]);
  locate(bhi[2], small[2], S.n_f[2], C.p[2], C.f[2]);
}

// record (entry) of cell C counted from the array start (cell (-1, -1, -1)); 24-bit
// multiplies (full rate) suffice: indices <= 448, strides <= 449 * 450
__device__ __forceinline__ unsigned int cell_index(const SceneDev& S, const Cell& C) {
  return (unsigned)C.p[0] + __umul24((unsigned)C.p[1], (unsigned)S.P0) + __umul24((unsigned)C.p[2], (unsigned)S.P01);
}

// Padded cell indices (p0, p1, p2) of record r: the inverse of cell_index, with the two
// divisions done as a multiply by a host-computed reciprocal and a shift (exact for
// r < 2^27, see the ABI).
__device__ __forceinline__ void cell_of_record(const SceneDev& S, unsigned r, int p[3]) {
  const unsigned t = (unsigned)(((unsigned long long)r * S.rec_div_m[0]) >> S.rec_div_s[0]);  // r / P0
  const unsigned z = (unsigned)(((unsigned long long)r * S.rec_div_m[1]) >> S.rec_div_s[1]);  // r / P01
  p[0] = (int)(r - t * (unsigned)S.P0);
  p[1] = (int)(t - z * (unsigned)S.P1);
  p[2] = (int)z;
}

// Trilinear value q and its grid-unit gradient from the cell's coefficients C (see
// corner_coefficients) at the fractions f = (u, v, w): 11 fused multiply-adds.
__device__ __forceinline__ void trilinear(const float C[8], const float f[3], float& q, float g[3]) {
  const float u = f[0], v = f[1], w = f[2];
  const float t1 = fmaf(w, C[7], C[3]);                  // C3 + w C7
  const float gu = fmaf(w, C[5], fmaf(v, t1, C[1]));      // C1 + v C3 + w C5 + v w C7
  const float t3 = fmaf(w, C[6], C[2]);                  // C2 + w C6
  const float t5 = fmaf(v, C[7], C[5]);                  // C5 + v C7
  const float t6 = fmaf(v, C[6], C[4]);                  // C4 + v C6
  g[0] = gu;
  g[1] = fmaf(u, t1, t3);
  g[2] = fmaf(u, t5, t6);
  q = fmaf(u, gu, fmaf(v, t3, fmaf(w, C[4], C[0])));
}

// Same, plus the mixed second derivatives H = (q_uv, q_uw, q_vw); q and g are computed with
// exactly the operations of trilinear.
__device__ __forceinline__ void trilinear_h(const float C[8], const float f[3], float& q, float g[3], float H[3]) {
  const float u = f[0], v = f[1], w = f[2];
  const float t1 = fmaf(w, C[7], C[3]);
  const float gu = fmaf(w, C[5], fmaf(v, t1, C[1]));
  const float t3 = fmaf(w, C[6], C[2]);
  const float t5 = fmaf(v, C[7], C[5]);
  const float t6 = fmaf(v, C[6], C[4]);
  g[0] = gu;
  g[1] = fmaf(u, t1, t3);
  g[2] = fmaf(u, t5, t6);
  q = fmaf(u, gu, fmaf(v, t3, fmaf(w, C[4], C[0])));
  H[0] = t1;                    // d2q / dx dy
  H[1] = t5;                    // d2q / dx dz
  H[2] = fmaf(u, C[7], C[6]);   // d2q / dy dz
}

// Force of Eq. (1) in code units from a cell's corner codes and the fractions:
// G_a = (1 + delta) dq/du_a; the grid-unit force is K_a = G_a km_a, km_a = dec / voxel_a^2
// (the Sharma step folds km_a into its stage coefficients).
__device__ __forceinline__ void force_code(const SceneDev& S, const float c[8], const float f[3], float G[3]) {
  float q, g[3];
  trilinear(c, f, q, g);
  float eta = fmaf(q, S.dec, S.one_plus_off);
#pragma unroll
  for (int a = 0; a < 3; ++a) G[a] = eta * g[a];
}

// Grid-unit force of Eq. (1) from a cell's corner codes and the fractions:
// K_a = (1 + delta) d(delta)/du_a / voxel_a^2.
__device__ __forceinline__ void force_of(const SceneDev& S, const float c[8], const float f[3], float K[3]) {
  float q, g[3];
  trilinear(c, f, q, g);
  float eta = fmaf(q, S.dec, S.one_plus_off);
#pragma unroll
  for (int a = 0; a < 3; ++a) K[a] = eta * (g[a] * S.km[a]);
}

template <int DT>
__device__ __forceinline__ void force_at_rec(const SceneDev& S, unsigned rec, const float f[3], float K[3]) {
  float c[8];
  fetch_cell<DT>(S, rec, c);
  force_of(S, c, f, K);
}

template <int DT>
__device__ __forceinline__ void force_at(const SceneDev& S, const Cell& C, float K[3]) {
  force_at_rec<DT>(S, cell_index(S, C), C.f, K);
}

// Sample recorder of sharma_step: called with the stage (0, 1, 2 for P1, P2, P3), the
// record index and the located cell of each of a step's three samples. The forward pass
// records nothing; the adjoint's replay keeps them for the reverse sweep.
struct NoRecord {
  __device__ __forceinline__ void operator()(int, unsigned, const Cell&) const {}
};

// Work issued by sharma_step right after the gather of its first sample (the forward's
// checkpoint stores): gfx9 counts loads and stores in one in-order counter, so stores
// issued before that gather would be waited for with it, while stores issued after it
// complete in the shadow of the step's arithmetic.
struct NoIssue {
  __device__ __forceinline__ void operator()() const {}
};

// ------------------------------------------------------------------------------------
// ray state in grid units: position = base(t) + d, velocity = V + e, where the base is
// the straight line through the entry point with the entry velocity V. The base is
// carried exactly: at half step j it is bh(j) + lo(j) with bh(j) = U0hi + j*g2hi a sum
// of multiples of 2^-14 (exact in binary32 while |u| < 512) and lo(j) = U0lo + j*g2lo.
// ------------------------------------------------------------------------------------
struct RayBase {
  float U0hi[3], U0lo[3], g2hi[3], g2lo[3];
  float V[3];  // entry velocity (m per unit t), binary32
};

__device__ __forceinline__ void split14(df x, float& hi, float& lo) {
  hi = rintf(x.hi * 16384.0f) * (1.0f / 16384.0f);
  lo = (x.hi - hi) + x.lo;
}

// entry velocity v0 = (1 + delta(x0)) dir (Sharma's |v| = eta) and the base increments
template <int DT>
__device__ __forceinline__ void make_base(const SceneDev& S, const Ray& R, RayBase& B, Cell& C0) {
  float bh[3], small[3];
  for (int a = 0; a < 3; ++a) {
    split14(R.U0[a], B.U0hi[a], B.U0lo[a]);
    bh[a] = B.U0hi[a];
    small[a] = B.U0lo[a];
  }
  locate3(S, bh, small, C0);
  float c[8];
  fetch_cell<DT>(S, cell_index(S, C0), c);
  float q, g[3];
  trilinear(c, C0.f, q, g);
  float delta = fmaf(q, S.dec, S.off);
  df eta0 = dd_fast(1.0f, delta);
  for (int a = 0; a < 3; ++a) {
    df v = dd_mul(eta0, R.dir[a]);
    B.V[a] = dd_to_f(v);
    df G2 = dd_mul_f(dd_mul(dd_mul(S.h, v), S.inv_vox[a]), 0.5f);
    split14(G2, B.g2hi[a], B.g2lo[a]);
  }
}

struct State {
  float bh[3];  // base hi at the start of the step (half step j = 2n)
  float jf;     // 2n as a float
  float d[3];   // position deviation (grid units)
  float e[3];   // velocity deviation (grid units per unit t)
  float pu[3];  // floor of u per axis at the position, unclamped, as sharma_step's last locate found it
};

__device__ __forceinline__ void state_at_step(const RayBase& B, int n, State& st) {
  st.jf = (float)(2 * n);
  for (int a = 0; a < 3; ++a) st.bh[a] = fmaf(st.jf, B.g2hi[a], B.U0hi[a]);
}

// small part of the position at half step (jf + dj) with deviation dev
__device__ __forceinline__ float small_part(const RayBase& B, int a, float jf, float dev) {
  return fmaf(jf, B.g2lo[a], B.U0lo[a]) + dev;
}

// Deviations (grid units) of the stage points of a Sharma step from the state's base
// point, given the stage forces in code units (G = K / km): P2 = x + h/2 v + h^2/8 K1,
// P3 = x + h v + h^2/2 K2, with x + h v shared with the position update. The adjoint's
// reverse relocates stage points with these same functions.
__device__ __forceinline__ float stage2_dev(const SceneDev& S, const State& st, int a, float G1) {
  return fmaf(S.c_p2[a], G1, fmaf(S.h_2, st.e[a], st.d[a]));
}
__device__ __forceinline__ float stage3_base(const SceneDev& S, const State& st, int a) {
  return fmaf(S.hf, st.e[a], st.d[a]);
}
__device__ __forceinline__ float stage3_dev(const SceneDev& S, int a, float base3, float G2) {
  return fmaf(S.c_p3[a], G2, base3);
}

// One Sharma step of Eq. (1) (grid units):
//   K1 = D(P1), P1 = x
//   K2 = D(P2), P2 = x + h/2 v + h^2/8 K1
//   K3 = D(P3), P3 = x + h v + h^2/2 K2
//   x <- x + h v + h^2/6 (K1 + 2 K2),  v <- v + h/6 (K1 + 4 K2 + K3)
// The base absorbs the h V part of every position. On return st holds the new state
// and `C` the located cell of the new position (the next step's first sample). With
// FULL false the step ends once its third sample is located and recorded (no force
// there, no new state): the last step of a replayed chunk needs only its samples.
template <int DT, class Record = NoRecord, class Issue = NoIssue, bool FULL = true>
__device__ __forceinline__ void sharma_step(const SceneDev& S, const RayBase& B, State& st, Cell& C,
                                            const Record& record = Record(), const Issue& issue = Issue()) {
  float G1[3], G2[3], G3[3], bh2[3], bh3[3], sm[3], base3[3];
  unsigned rec = cell_index(S, C);
  record(0, rec, C);
  {
    float c[8];
    fetch_cell<DT>(S, rec, c);
    __builtin_amdgcn_sched_barrier(0);
    issue();
    __builtin_amdgcn_sched_barrier(0);
    force_code(S, c, C.f, G1);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    bh2[a] = st.bh[a] + B.g2hi[a];
    sm[a] = small_part(B, a, st.jf + 1.0f, stage2_dev(S, st, a, G1[a]));
  }
  locate3(S, bh2, sm, C);
  rec = cell_index(S, C);
  record(1, rec, C);
  {
    float c[8];
    fetch_cell<DT>(S, rec, c);
    force_code(S, c, C.f, G2);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    bh3[a] = bh2[a] + B.g2hi[a];
    base3[a] = stage3_base(S, st, a);
    sm[a] = small_part(B, a, st.jf + 2.0f, stage3_dev(S, a, base3[a], G2[a]));
  }
  locate3(S, bh3, sm, C);
  rec = cell_index(S, C);
  record(2, rec, C);
  if constexpr (!FULL) return;
  {
    float c[8];
    fetch_cell<DT>(S, rec, c);
    force_code(S, c, C.f, G3);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float dn = fmaf(S.c_x[a], fmaf(2.0f, G2[a], G1[a]), base3[a]);
    float en = fmaf(S.c_v[a], fmaf(4.0f, G2[a], G1[a]) + G3[a], st.e[a]);
    st.d[a] = dn;
    st.e[a] = en;
    st.bh[a] = bh3[a];
  }
  st.jf += 2.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    locate_floor(st.bh[a], small_part(B, a, st.jf, st.d[a]), S.n_f[a], C.p[a], C.f[a], st.pu[a]);
}

// One quasi-linear step (Sec. 2.B): the forces are taken on the straight entry line, at
// its half-step points j = 2n, 2n + 1, 2n + 2 (exact base plus its small part, no
// deviation), and drive the same update as sharma_step. Kc carries the force at the
// step's start point, which the previous step computed as its end point.
template <int DT>
__device__ __forceinline__ void ql_step(const SceneDev& S, const RayBase& B, State& st, float Kc[3]) {
  float K2[3], K3[3], bh2[3], bh3[3], sm[3];
  Cell C;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    bh2[a] = st.bh[a] + B.g2hi[a];
    sm[a] = small_part(B, a, st.jf + 1.0f, 0.0f);
  }
  locate3(S, bh2, sm, C);
  force_at<DT>(S, C, K2);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    bh3[a] = bh2[a] + B.g2hi[a];
    sm[a] = small_part(B, a, st.jf + 2.0f, 0.0f);
  }
  locate3(S, bh3, sm, C);
  force_at<DT>(S, C, K3);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float dn = st.d[a] + fmaf(S.hf, st.e[a], S.h2_6 * fmaf(2.0f, K2[a], Kc[a]));
    float en = st.e[a] + S.h_6 * (fmaf(4.0f, K2[a], Kc[a]) + K3[a]);
    st.d[a] = dn;
    st.e[a] = en;
    st.bh[a] = bh3[a];
    Kc[a] = K3[a];
  }
  st.jf += 2.0f;
}

// Position strictly outside the box on some axis (or not a number).
__device__ __forceinline__ bool outside_box(const SceneDev& S, const RayBase& B, const State& st) {
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float sm = small_part(B, a, st.jf, st.d[a]);
    float lo_gap = (st.bh[a] - 0.5f) + sm;            // u - 1/2, first term exact
    float hi_gap = (st.bh[a] - S.hi_bound[a]) + sm;   // u - (n + 1/2), first term exact
    inside = inside & (lo_gap >= 0.0f) & (hi_gap <= 0.0f);
  }
  return !inside;
}

// The same test after a sharma_step, from its last locate (C, st.pu): u = pu + f lies in
// [1/2, n + 1/2] iff -pu <= f - 1/2 <= n - pu, where both bounds are exact integers and
// f - 1/2 has the sign of the exact difference; NaN (a non-finite position) is outside.
__device__ __forceinline__ bool outside_located(const SceneDev& S, const State& st, const Cell& C) {
  bool inside = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float g = C.f[a] - 0.5f;
    inside = inside & (g >= -st.pu[a]) & (g <= S.n_f[a] - st.pu[a]);
  }
  return !inside;
}

// A non-finite component makes the sum non-finite (inf - inf is NaN); the deviations
// stay within a few hundred grid units, so the sum of finite ones cannot overflow.
__device__ __forceinline__ bool state_finite(const State& st) {
  return isfinite(((st.d[0] + st.d[1]) + (st.d[2] + st.e[0])) + (st.e[1] + st.e[2]));
}

// Deviation of the wall hit from the undeflected hit, from the last state:
// x = base + d, v = V + e (metres). With b = V.n, s_b the base point's distance to the
// wall along V, the hit is x + s v with s = s_b - (d.n + s_b e.n) / (b + e.n), and
// X - X0 = d + (s - s_b) V + s e. Returns false when v does not face the wall.
__device__ __forceinline__ bool wall_deflection(const SceneDev& S, const RayBase& B, const State& st, float dX[3],
                                                float* s_out) {
  float dm[3], em[3], Rb[3];
  float b = 0.0f, dn = 0.0f, en = 0.0f, wb = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dm[a] = st.d[a] * S.vox[a];
    em[a] = st.e[a] * S.vox[a];
    float u = st.bh[a] + fmaf(st.jf, B.g2lo[a], B.U0lo[a]);
    Rb[a] = S.lo_f[a] + (u - 0.5f) * S.vox[a];
    b += B.V[a] * S.wall_n_f[a];
    dn += dm[a] * S.wall_n_f[a];
    en += em[a] * S.wall_n_f[a];
    wb += (S.wall_org_f[a] - Rb[a]) * S.wall_n_f[a];
  }
  if (!(b + en < 0.0f)) return false;
  float sb = wb / b;
  float ds = -(dn + sb * en) / (b + en);
  float s = sb + ds;
#pragma unroll
  for (int a = 0; a < 3; ++a) dX[a] = dm[a] + ds * B.V[a] + s * em[a];
  if (s_out) *s_out = s;
  return true;
}

}  // namespace rbos

namespace rbos {

// ------------------------------------------------------------------------------------
// wavefront reductions (DPP within rows, row broadcasts across them; all 64 lanes must
// be active). The result is returned to every lane.
// ------------------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(dpp_i<CTRL, ROW_MASK>(__float_as_int(v)));
}

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<0xb1>(v);        // quad_perm [1,0,3,2]
  v += dpp_f<0x4e>(v);        // quad_perm [2,3,0,1]
  v += dpp_f<0x141>(v);       // row_half_mirror
  v += dpp_f<0x140>(v);       // row_mirror
  v += dpp_f<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// max over lanes of a non-negative int
__device__ __forceinline__ int wave_max_nonneg(int v) {
  v = max(v, dpp_i<0xb1>(v));
  v = max(v, dpp_i<0x4e>(v));
  v = max(v, dpp_i<0x141>(v));
  v = max(v, dpp_i<0x140>(v));
  v = max(v, dpp_i<0x142, 0xa>(v));
  v = max(v, dpp_i<0x143, 0xc>(v));
  return __builtin_amdgcn_readlane(v, 63);
}

}  // namespace rbos

namespace rbos {

// ------------------------------------------------------------------------------------
// per-ray header stored with the checkpoints (component-major, n_rays per component):
// the straight-line base (U0hi, U0lo, g2hi, g2lo), the entry velocity V, the final
// velocity deviation e and the wall distance parameter s of the last state. The adjoint
// reads it instead of redoing the double-float ray setup.
// ------------------------------------------------------------------------------------
constexpr int RAY_HEADER = 19;

__device__ __forceinline__ void store_ray_header(const SceneDev& S, int r, const RayBase& B, const State& st,
                                                 float s) {
  float* p = S.ckpt + (size_t)r;
  const size_t P = (size_t)S.ckpt_pad;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gst_stream(p + (0 + a) * P, B.U0hi[a]);
    gst_stream(p + (3 + a) * P, B.U0lo[a]);
    gst_stream(p + (6 + a) * P, B.g2hi[a]);
    gst_stream(p + (9 + a) * P, B.g2lo[a]);
    gst_stream(p + (12 + a) * P, B.V[a]);
    gst_stream(p + (15 + a) * P, st.e[a]);
  }
  gst_stream(p + 18 * P, s);
}

__device__ __forceinline__ void load_ray_header(const SceneDev& S, int r, RayBase& B, float e_end[3], float& s) {
  const float* p = S.ckpt + (size_t)r;
  const size_t P = (size_t)S.ckpt_pad;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    B.U0hi[a] = gld(p + (0 + a) * P);
    B.U0lo[a] = gld(p + (3 + a) * P);
    B.g2hi[a] = gld(p + (6 + a) * P);
    B.g2lo[a] = gld(p + (9 + a) * P);
    B.V[a] = gld(p + (12 + a) * P);
    e_end[a] = gld(p + (15 + a) * P);
  }
  s = gld(p + 18 * P);
}

}  // namespace rbos
