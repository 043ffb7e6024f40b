// trace_adj.hip -- Sec. 2.D: exact gradient of L_BOS with respect to eta - 1 per voxel,
// back-propagated through the wall step and every Sharma step of Eq. (1).
//
// Per wavefront (64 rays of one tile), segments between checkpoints are processed from
// the last to the first, aligned on the step index so that the tile's rays move through
// the same cells together. A segment is replayed forward from its checkpoint in chunks
// of KS steps, keeping in LDS either each step's start state (then the reverse relocates
// the step's samples) or, for strides 3 and 4 (a segment is then one chunk), the cells
// and fractions of its three samples; the chunk is then reversed step by step. Each
// sample's contributions are merged per lane, as monomial coefficients, while the ray
// stays in one cell; lanes that left the same cell are summed across the wavefront into a
// per-wavefront LDS cache of cell totals, which goes to the gradient with one FP64 atomic
// per corner. A wavefront lowers its issue priority while replaying and raises it while
// merging. Most loops stay rolled so the kernel fits the instruction cache; the per-ray
// geometry comes from the header the forward pass stored with the checkpoints.
#include <climits>

#include "rbos_device.hpp"
#include "rbos_launch.hpp"

namespace rbos {

// Everything the reverse sweep needs about one sample.
struct SampleRev {
  float f[3];        // fraction within the cell
  int key;           // record index of the cell (cell_index)
  float g[3], H[3];  // code-unit gradient and mixed second derivatives
  float eta;         // 1 + delta
};

// A sample from its cell's 8 corner codes, record index and fractions.
__device__ __forceinline__ void sample_rev_at(const SceneDev& S, const float c[8], unsigned rec, const float f[3],
                                              SampleRev& R) {
  float q;
  trilinear_h(c, f, q, R.g, R.H);
  R.eta = fmaf(q, S.dec, S.one_plus_off);
#pragma unroll
  for (int a = 0; a < 3; ++a) R.f[a] = f[a];
  R.key = (int)rec;
}

template <int DT>
__device__ __forceinline__ void sample_rev(const SceneDev& S, const Cell& C, SampleRev& R) {
  float c[8];
  const unsigned rec = cell_index(S, C);
  fetch_cell<DT>(S, rec, c);
  sample_rev_at(S, c, rec, C.f, R);
}

// Reverse of G = force_code(P) (code units, G_a = eta dq/du_a) for its adjoint
// w = dL/dG: returns p = dL/dP (grid units) and adds the sample's contributions to
// dL/d(delta_c) for the 8 corners of its cell, times dec, to acc:
//   s = dec sum_a w_a g_a,  W_a = eta w_a,
//   p_b = s g_b + sum_{a != b} W_a H_ab,
//   dec dL/d delta_c = s w_c + sum_a W_a dw_c/du_a,
// with w_c the trilinear weight of corner c. The contributions are multilinear in the
// fractions (u, v, w) = f, so they are kept as the coefficients of the 8 monomials
// m = u^(m & 1) v^(m >> 1 & 1) w^(m >> 2): s m + sum_a W_a dm/du_a. Samples in one cell
// share the monomials' frame, so their coefficients add up; corner values follow from
// the totals (corner_of_monomials, scaled by 1 / dec). In apron cells the field is
// constant along the clamped axis (g and H vanish there); the two corners that share one
// edge voxel receive contributions that add up to the clamped-axis weights.
__device__ __forceinline__ void force_rev(const SceneDev& S, const SampleRev& R, const float w[3], float p[3],
                                          float acc[8]) {
  const float s = S.dec * fmaf(w[0], R.g[0], fmaf(w[1], R.g[1], w[2] * R.g[2]));
  const float Wx = R.eta * w[0], Wy = R.eta * w[1], Wz = R.eta * w[2];
  // H = (H_xy, H_xz, H_yz)
  p[0] = fmaf(s, R.g[0], fmaf(Wy, R.H[0], Wz * R.H[1]));
  p[1] = fmaf(s, R.g[1], fmaf(Wx, R.H[0], Wz * R.H[2]));
  p[2] = fmaf(s, R.g[2], fmaf(Wx, R.H[1], Wy * R.H[2]));
  const float u = R.f[0], v = R.f[1], x = R.f[2];
  const float m1 = fmaf(s, u, Wx);              // u:   s u + Wx
  const float m2 = fmaf(s, v, Wy);              // v:   s v + Wy
  const float m3 = fmaf(v, m1, Wy * u);         // uv:  s uv + Wx v + Wy u
  acc[0] += s;                                  // 1
  acc[1] += m1;
  acc[2] += m2;
  acc[3] += m3;
  acc[4] += fmaf(s, x, Wz);                     // w:   s w + Wz
  acc[5] = fmaf(x, m1, fmaf(Wz, u, acc[5]));    // uw:  s uw + Wx w + Wz u
  acc[6] = fmaf(x, m2, fmaf(Wz, v, acc[6]));    // vw:  s vw + Wy w + Wz v
  acc[7] = fmaf(x, m3, fmaf(Wz, u * v, acc[7]));  // uvw: s uvw + Wx vw + Wy uw + Wz uv
}

// Corner c of a cell from its 8 monomial totals: the trilinear weight of corner
// (i, j, k) is the product over the axes of (1 - u) (bit 0) or u (bit 1), so monomial m
// enters corner c when it holds every axis set in c, with the sign (-1) per axis it holds
// beyond c. Summed in FP64.
__device__ __forceinline__ double corner_of_monomials(const float* vals, int c) {
  double g = 0.0;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    if ((m & c) == c) {
      const double t = (double)vals[m];
      g += (__popc(m & ~c) & 1) ? -t : t;
    }
  }
  return g;
}

// Per-lane merge of the samples' monomial coefficients by cell. A lane that leaves a cell
// parks its sums. With PARK (kernels with registers to spare), the parked sums of a cell
// are reduced across the wavefront when one of its lanes leaves a second cell (its park
// is needed again), together with those of every other lane parked in that cell: the
// tile's rays leave a cell over a few samples, so one reduction then covers most of them.
// Without, the lanes leaving cells at a sample are reduced at once.
constexpr int CELL_NONE = INT_MIN;

struct Accum {
  float acc[8];
  int key;        // record index of the cell (< 2^27), CELL_NONE when empty
  float park[8];  // the sums of the last cell left
  int pkey;       // its record index, CELL_NONE when the park is free
};

__device__ __forceinline__ void accum_init(Accum& A) {
#pragma unroll
  for (int k = 0; k < 8; ++k) A.acc[k] = A.park[k] = 0.0f;
  A.key = A.pkey = CELL_NONE;
}

// Sum 8 per-lane values over the 64 lanes, all eight at once: each exchange step halves
// the lanes per value and keeps the values apart (permlane32 / permlane16 swaps between
// value pairs, then one row rotation by 8), and the last three steps reduce within
// groups of 8 lanes. On return every lane of group g = lane / 8 holds the total of value
// (g & 4) | (g & 1) << 1 | (g >> 1) & 1. All 64 lanes must be active.
__device__ __forceinline__ float wave_sum8(const float v[8]) {
  float w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k + 4]), false, false);
    w[k] = __uint_as_float(s[0]) + __uint_as_float(s[1]);  // lanes 0-31: value k, 32-63: value k + 4
  }
  float u[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(w[2 * k]), __float_as_uint(w[2 * k + 1]), false, false);
    u[k] = __uint_as_float(s[0]) + __uint_as_float(s[1]);  // 16-lane rows: values 2k, 2k+1, 2k+4, 2k+5
  }
  const float t0 = u[0] + dpp_f<0x128>(u[0]);  // row_ror:8
  const float t1 = u[1] + dpp_f<0x128>(u[1]);
  float z = (__lane_id() & 8) ? t1 : t0;
  z += dpp_f<0xb1>(z);   // quad_perm [1,0,3,2]
  z += dpp_f<0x4e>(z);   // quad_perm [2,3,0,1]
  z += dpp_f<0x141>(z);  // row_half_mirror: completes the sum over 8 lanes
  return z;
}

// Per-wavefront cache of cell totals between the wavefront reduction and the FP64
// atomics: a cell is left by the tile's rays over several steps (the bundle crosses a
// face obliquely), so its partial totals are merged here and reach the gradient once.
// Slot p holds 8 corner totals in LDS (corner a + 2b + 4c) and its key in lane p of one
// register. Slots are written out in batches every few chunks (those not touched since
// the last batch) and at the end of the tile, so the atomics' latency is exposed once per
// batch rather than once per cell (a non-returning atomic still counts in vmcnt, which the
// next load waits on). A miss with every slot taken writes one slot out at once.
// The slot masks are 32-bit (one scalar register each): the kernels run at the scalar
// register limit, and every register freed spares a reload of a scene constant.
constexpr int PEND_SLOTS = 32;
static_assert(PEND_SLOTS == 32, "slot masks are one 32-bit word, all of whose bits are slots");

struct Pending {
  float* vals;        // LDS, PEND_SLOTS * 8 floats, wave-private
  int key;            // lane p < PEND_SLOTS: key of slot p; CELL_NONE when free (always for p >= PEND_SLOTS)
  int next;           // wave-uniform: slot replaced when all are taken
  unsigned occupied;  // wave-uniform slot masks
  unsigned touched;   // slots hit or filled since the last batch write-out
};

__device__ __forceinline__ double* voxel_of_corner(const SceneDev& S, int key, int c) {
  int p[3];
  cell_of_record(S, (unsigned)key, p);
  // apron corners map to the edge voxel they repeat
  const int x = min(max(p[0] - 1 + (c & 1), 0), S.n[0] - 1);
  const int y = min(max(p[1] - 1 + ((c >> 1) & 1), 0), S.n[1] - 1);
  const int z = min(max(p[2] - 1 + (c >> 2), 0), S.n[2] - 1);
  return &S.grad[((size_t)z * S.n[1] + y) * S.n[0] + x];
}

// Order this lane's LDS accesses of the cache against other lanes' (the hardware runs a
// wavefront's LDS instructions in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Corner of the total that lane group g = lane / 8 holds after wave_sum8.
__device__ __forceinline__ int group_corner(int lane) {
  const int g = lane >> 3;
  return (g & 4) | ((g & 1) << 1) | ((g >> 1) & 1);
}

// Add the 8 wavefront totals of cell `key` (wave_sum8's layout) to its slot, taking a
// free slot, or writing one out, when the cell has none.
__device__ __forceinline__ void cache_add(const SceneDev& S, Pending& P, int key, float total, int lane) {
  const int corner = group_corner(lane);
  const unsigned hit = (unsigned)__ballot(P.key == key);  // only lanes < PEND_SLOTS hold keys
  int slot;
  if (hit) {
    slot = __ffs((int)hit) - 1;
    if ((lane & 7) == 0) atomicAdd(&P.vals[slot * 8 + corner], total);
  } else {
    const unsigned freem = ~P.occupied;
    if (freem) {
      slot = __ffs((int)freem) - 1;
    } else {
      slot = P.next;
      P.next = (P.next + 1) & (PEND_SLOTS - 1);
      const int old = __builtin_amdgcn_readlane(P.key, slot);
      if (lane < 8)
        gatomic_add(voxel_of_corner(S, old, lane), corner_of_monomials(P.vals + slot * 8, lane) * S.inv_dec_d);
      wave_lds_order();
    }
    if ((lane & 7) == 0) P.vals[slot * 8 + corner] = total;
    if (lane == slot) P.key = key;
    P.occupied |= 1u << slot;
  }
  P.touched |= 1u << slot;
  wave_lds_order();
}

// Add the accumulators of lanes with `sel` to the cache (lanes that hold the same cell
// summed across the wavefront) and restart them. Must run with all 64 lanes active.
__device__ __forceinline__ void flush(const SceneDev& S, Accum& A, bool sel, int lane, Pending& P) {
  unsigned long long pend = __ballot(sel);
  while (pend) {
    const int leader = __ffsll((long long)pend) - 1;
    const int key = __builtin_amdgcn_readlane(A.key, leader);
    const bool mine = sel && A.key == key;
    const unsigned long long mine_m = __ballot(A.key == key);  // a single comparison: no VALU round trip
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = mine ? A.acc[k] : 0.0f;
    cache_add(S, P, key, wave_sum8(v), lane);
    pend &= ~mine_m;
  }
  if (sel) {
#pragma unroll
    for (int k = 0; k < 8; ++k) A.acc[k] = 0.0f;
  }
}

// For every cell parked by a lane with `trig`: the parks of all lanes holding that cell
// go to the cache, summed across the wavefront, and are freed. Must run with all 64
// lanes active.
__device__ __forceinline__ void flush_parks(const SceneDev& S, Accum& A, bool trig, int lane, Pending& P) {
  unsigned long long pend = __ballot(trig);
  while (pend) {
    const int leader = __ffsll((long long)pend) - 1;
    const int key = __builtin_amdgcn_readlane(A.pkey, leader);
    const bool mine = A.pkey == key;
    const unsigned long long mine_m = __ballot(A.pkey == key);  // taken before the pkey reset below
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = mine ? A.park[k] : 0.0f;
    cache_add(S, P, key, wave_sum8(v), lane);
    pend &= ~mine_m;
    if (mine) A.pkey = CELL_NONE;
  }
}

// Write the slots in `which` out to the gradient and free them.
__device__ __forceinline__ void write_out(const SceneDev& S, Pending& P, unsigned which, int lane) {
  wave_lds_order();
#pragma unroll 1
  for (int q = 0; q < PEND_SLOTS * 8 / 64; ++q) {
    if (((which >> (8 * q)) & 0xffu) == 0) continue;
    const int idx = q * 64 + lane, slot = idx >> 3;
    const int key = __shfl(P.key, slot);
    if ((which >> slot) & 1u)
      gatomic_add(voxel_of_corner(S, key, idx & 7), corner_of_monomials(P.vals + slot * 8, idx & 7) * S.inv_dec_d);
  }
  wave_lds_order();
  if (lane < PEND_SLOTS && ((which >> lane) & 1u)) P.key = CELL_NONE;
  P.occupied &= ~which;
}

// Batch write-out: the slots not touched since the last one (cells the rays have left).
__device__ __forceinline__ void chunk_end(const SceneDev& S, Pending& P, int lane) {
  const unsigned stale = P.occupied & ~P.touched;
  if (stale) write_out(S, P, stale, lane);
  P.touched = 0;
}

// Lanes with act take a sample in cell `key`: a lane that enters a new cell parks the sums
// of the one it leaves (after its park has been flushed, if taken), or flushes them
// without PARK, and starts from zero. The caller then adds the sample to A.acc. act_m is
// the ballot of act, which the caller takes once for all stages of a step. The wave-uniform
// tests combine ballots of single comparisons in scalar registers: a ballot of a compound
// lane predicate is lowered through a VALU select and compare, on the latency path of
// every sample.
template <bool PARK>
__device__ __forceinline__ void enter(const SceneDev& S, Accum& A, bool act, unsigned long long act_m, int key,
                                      int lane, Pending& P) {
  const bool out = act && key != A.key && A.key != CELL_NONE;
  const unsigned long long out_m = act_m & __ballot(key != A.key) & __ballot(A.key != CELL_NONE);
  if (out_m) {
    __builtin_amdgcn_s_setprio(3);  // the merge's reduction chains first (see the recording form)
    if (PARK) {
      const bool busy = out && A.pkey != CELL_NONE;
      const unsigned long long busy_m = out_m & __ballot(A.pkey != CELL_NONE);
      if (busy_m) flush_parks(S, A, busy, lane, P);
      if (out) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          A.park[k] = A.acc[k];
          A.acc[k] = 0.0f;
        }
        A.pkey = A.key;
      }
    } else {
      flush(S, A, out, lane, P);
    }
    __builtin_amdgcn_s_setprio(1);
  }
  if (act) A.key = key;
}

// Merge a sample's monomial coefficients ct (lanes with act) into the accumulators.
template <bool PARK>
__device__ __forceinline__ void accumulate(const SceneDev& S, Accum& A, bool act, int key, const float ct[8],
                                           int lane, Pending& P) {
  enter<PARK>(S, A, act, __ballot(act), key, lane, P);
  if (act) {
#pragma unroll
    for (int k = 0; k < 8; ++k) A.acc[k] += ct[k];
  }
}

// Tile end: the parks, then the open accumulators, into the cache; every slot out.
__device__ __forceinline__ void drain(const SceneDev& S, Accum& A, Pending& P, int lane) {
  if (__ballot(A.pkey != CELL_NONE)) flush_parks(S, A, A.pkey != CELL_NONE, lane, P);
  flush(S, A, A.key != CELL_NONE, lane, P);
  if (P.occupied) write_out(S, P, P.occupied, lane);
}

__device__ __forceinline__ void load_ckpt(const SceneDev& S, int r, int slot, State& st) {
  const float* ck = S.ckpt + (size_t)(RAY_HEADER + slot * 6) * (size_t)S.ckpt_pad + (size_t)r;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    st.d[a] = gld(ck + (size_t)a * S.ckpt_pad);
    st.e[a] = gld(ck + (size_t)(3 + a) * S.ckpt_pad);
  }
}

__device__ __forceinline__ void locate_state(const SceneDev& S, const RayBase& B, const State& st, Cell& C) {
  float sm[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) sm[a] = small_part(B, a, st.jf, st.d[a]);
  locate3(S, st.bh, sm, C);
}

// Occupancy: chunks of 8 steps take 13 KB of LDS per wavefront, so 3 wavefronts per SIMD;
// chunks of 6 take 10 KB, and 4 fit when the registers are held to 128.
template <int KS>
constexpr int adj_waves_per_simd() { return KS == 6 ? 4 : 3; }

// Recording form: chunks of 4 steps take 13 KB of LDS per wavefront (3 wavefronts per
// SIMD), chunks of 3 take 10 KB (4 per SIMD with the registers held to 128).
template <int KS>
constexpr int rec_waves_per_simd() { return KS == 3 ? 4 : 3; }

// LDS per wavefront: the replayed step-start states of one chunk, slot (i, component) of
// lane l at replay[(i * 6 + c) * 64 + l] (conflict-free), then the cell-total cache.
template <int KS>
constexpr int lds_floats_per_wave() { return KS * 6 * 64 + PEND_SLOTS * 8; }

// Ray setup of the adjoint: the ray of this lane, its step count and whether it carries
// a gradient, its straight-line base from the header, and the adjoint of the last state
// through the wall step X = x + s v:
//   lambda_x = lambda_X - n (v . lambda_X)/(v . n),  lambda_v = s lambda_x
// (metres; grid units multiply by the voxel size), returned as rb = dL/dd, tb = dL/de.
struct AdjRay {
  int r, q, n;  // ray, its checkpoint entry, its step count
  bool active;
  RayBase B;
  float rb[3], tb[3];
};

__device__ __forceinline__ void adjoint_ray_setup(const SceneDev& S, int tile, int lane, AdjRay& R) {
  int pix = 0;
  R.r = 0;
  R.q = 0;
  R.n = 0;
  R.active = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) R.rb[a] = R.tb[a] = 0.0f;
  int smp;
  if (!tile_ray(S, tile, lane, R.r, pix, smp)) return;
  const int r = R.r;
  R.q = ckpt_entry(S, r, pix, smp);
  R.n = gld(S.n_steps + r);
  const unsigned char st = gld(S.status + r);
  const float lu = gld(S.adj_dL_duv + 2 * (size_t)r), lv = gld(S.adj_dL_duv + 2 * (size_t)r + 1);
  float ld[3] = {0.0f, 0.0f, 0.0f};  // dL/d(unit direction at the wall)
  if (S.adj_dL_ddir) {
#pragma unroll
    for (int a = 0; a < 3; ++a) ld[a] = gld(S.adj_dL_ddir + 3 * (size_t)r + a);
  }
  const bool seed = !(lu == 0.0f && lv == 0.0f) || !(ld[0] == 0.0f && ld[1] == 0.0f && ld[2] == 0.0f);
  R.active = R.n > 0 && !(st & (RAY_NO_WALL_HIT | RAY_NONFINITE | RAY_MISSED_BOX)) && seed;
  if (!R.active) return;
  float e_end[3], s;
  load_ray_header(S, R.q, R.B, e_end, s);
  float v[3], lX[3], vn = 0.0f, vl = 0.0f, v2 = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    v[a] = R.B.V[a] + e_end[a] * S.vox[a];
    lX[a] = lu * S.wall_u_f[a] + lv * S.wall_v_f[a];
    vn += v[a] * S.wall_n_f[a];
    vl += v[a] * lX[a];
    v2 += v[a] * v[a];
  }
  const float qv = vl / vn;
  // the direction v / |v| at the wall: its adjoint (ld - d (d . ld)) / |v| joins dL/dv
  const float inv_v = 1.0f / sqrtf(v2);
  const float dl = (v[0] * ld[0] + v[1] * ld[1] + v[2] * ld[2]) * inv_v;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float lx = lX[a] - S.wall_n_f[a] * qv;
    const float lvd = (ld[a] - v[a] * inv_v * dl) * inv_v;
    R.rb[a] = lx * S.vox[a];
    R.tb[a] = fmaf(lvd, S.vox[a], s * R.rb[a]);
  }
}

// Initial condition v0 = (1 + delta(x0)) dir: dL/d delta_c += w_c(x0) sum_a tb0_a dir_a /
// voxel_a, with tb0 = dL/dv0 in grid units and V = v0 (m per unit t). Contributions of
// lanes with `active`.
template <bool PARK>
__device__ __forceinline__ void entry_term(const SceneDev& S, const RayBase& B, const float V[3], bool active,
                                           const float tb0[3], Accum& A, Pending& P, int lane) {
  int key0 = 0;
  float c0v[8];
  if (active) {
    Cell C0;
    locate3(S, B.U0hi, B.U0lo, C0);
    const float vn = sqrtf(V[0] * V[0] + V[1] * V[1] + V[2] * V[2]);
    float kap = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) kap = fmaf(tb0[a], (V[a] / vn) * dd_to_f(S.inv_vox[a]), kap);
    kap *= S.dec;  // the accumulators hold dec times the contributions
    // kap w_c(x0) as monomial coefficients: kap m(f)
    const float u = C0.f[0], v = C0.f[1], w = C0.f[2];
    c0v[0] = kap;
    c0v[1] = kap * u;
    c0v[2] = kap * v;
    c0v[3] = c0v[1] * v;
    c0v[4] = kap * w;
    c0v[5] = c0v[1] * w;
    c0v[6] = c0v[2] * w;
    c0v[7] = c0v[3] * w;
    key0 = (int)cell_index(S, C0);
  }
  accumulate<PARK>(S, A, active, key0, c0v, lane, P);
}

// Reverse of one Sharma step for the state adjoints rb = dL/dd, tb = dL/de after it.
// The step (code-unit stage forces G_i at P_i, forward coefficients c_x, c_v, c_p2, c_p3)
//   P2 = x + h/2 e + c_p2 G1,  P3 = x + h e + c_p3 G2,
//   d' = x + h e + c_x (G1 + 2 G2),  e' = e + c_v (G1 + 4 G2 + G3)
// gives the force adjoints wC = dL/dG3 = c_v tb, wB = dL/dG2 = 2 c_x rb + 4 c_v tb +
// c_p3 p3, wA = dL/dG1 = c_x rb + c_v tb + c_p2 p2 (p_i = dL/dP_i from the stage's
// force_rev), and before the step rb + p3 + p2 + p1 and tb + h (rb + p3) + h/2 p2.
// stage_weights starts wA and wB from the step-end adjoints.
__device__ __forceinline__ void stage_weights(const SceneDev& S, const float rb[3], const float tb[3], float wA[3],
                                              float wB[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    wA[a] = fmaf(S.c_x[a], rb[a], S.c_v[a] * tb[a]);
    wB[a] = fmaf(S.c_x2[a], rb[a], S.c_v4[a] * tb[a]);
  }
}

// Stages C, B, A of the reverse (lanes with act), each sample's contributions into the
// accumulators of its cell; rb, tb become the adjoints before the step.
template <bool PARK>
__device__ __forceinline__ void reverse_stages(const SceneDev& S, Accum& A, Pending& P, bool act,
                                               const SampleRev& R1, const SampleRev& R2, const SampleRev& R3,
                                               float wA[3], float wB[3], float rb[3], float tb[3], int lane) {
  float rs[3], ts[3];
  const unsigned long long act_m = __ballot(act);
  enter<PARK>(S, A, act, act_m, act ? R3.key : 0, lane, P);
  if (act) {  // stage C
    float w[3], p[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = S.c_v[a] * tb[a];
    force_rev(S, R3, w, p, A.acc);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      rs[a] = rb[a] + p[a];
      ts[a] = fmaf(S.hf, rs[a], tb[a]);
      wB[a] = fmaf(S.c_p3[a], p[a], wB[a]);
    }
  }
  enter<PARK>(S, A, act, act_m, act ? R2.key : 0, lane, P);
  if (act) {  // stage B
    float p[3];
    force_rev(S, R2, wB, p, A.acc);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      rs[a] += p[a];
      ts[a] = fmaf(S.h_2, p[a], ts[a]);
      wA[a] = fmaf(S.c_p2[a], p[a], wA[a]);
    }
  }
  enter<PARK>(S, A, act, act_m, act ? R1.key : 0, lane, P);
  if (act) {  // stage A
    float p[3];
    force_rev(S, R1, wA, p, A.acc);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      rb[a] = rs[a] + p[a];
      tb[a] = ts[a];
    }
  }
}

template <int DT, int KS, bool STORED>
__device__ __forceinline__ void adjoint_tile(const SceneDev& S, int tile, int lane, float* __restrict__ replay) {
  constexpr bool PARK = adj_waves_per_simd<KS>() == 3;  // registers for the parks
  AdjRay R;
  adjoint_ray_setup(S, tile, lane, R);
  const int q = R.q, n = R.n;
  const bool active = R.active;
  const RayBase& B = R.B;
  float* rb = R.rb;
  float* tb = R.tb;
  // STORED (stride 1): every step's start state is in the checkpoints and a chunk is
  // filled from them; otherwise a segment of K steps is replayed from its checkpoint in
  // chunks.
  const int K = S.ckpt_k;
  const int seg_len = STORED ? KS : K;
  const int m_chunks = seg_len / KS;
  const int nseg_lane = active ? (n + seg_len - 1) / seg_len : 0;
  const int nseg = wave_max_nonneg(nseg_lane);

  Accum A;
  accum_init(A);
  Pending P{replay + KS * 6 * 64, CELL_NONE, 0, 0u, 0u};

  for (int seg = nseg - 1; seg >= 0; --seg) {
    for (int ch = m_chunks - 1; ch >= 0; --ch) {
      const int c0 = seg * seg_len + ch * KS;  // first step of the chunk
      const bool lane_chunk = active && c0 < n;
      if (STORED && lane_chunk) {
        // step j starts from slot j - 1 (zero deviation at j = 0); all loads first
        float v[KS][6];
#pragma unroll
        for (int i = 0; i < KS; ++i) {
          const int j = c0 + i;
          State st;
          if (j >= 1 && j < n) {
            load_ckpt(S, q, j - 1, st);
          } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) { st.d[a] = 0.0f; st.e[a] = 0.0f; }
          }
#pragma unroll
          for (int a = 0; a < 3; ++a) { v[i][a] = st.d[a]; v[i][3 + a] = st.e[a]; }
        }
#pragma unroll
        for (int i = 0; i < KS; ++i) {
#pragma unroll
          for (int c = 0; c < 6; ++c) replay[(i * 6 + c) * 64 + lane] = v[i][c];
        }
      } else if (!STORED && lane_chunk) {
        State st;
        Cell C;
        state_at_step(B, seg * K, st);
        if (seg == 0) {
#pragma unroll
          for (int a = 0; a < 3; ++a) { st.d[a] = 0.0f; st.e[a] = 0.0f; }
        } else {
          load_ckpt(S, q, seg - 1, st);
        }
        locate_state(S, B, st, C);
#pragma unroll 1
        for (int i = 0; i < ch * KS; ++i) sharma_step<DT>(S, B, st, C);  // to the chunk start
        const int cnt = min(KS, n - c0);  // steps of the chunk (the state after the last is not needed)
#pragma unroll 1
        for (int i = 0;; ++i) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            replay[(i * 6 + a) * 64 + lane] = st.d[a];
            replay[(i * 6 + 3 + a) * 64 + lane] = st.e[a];
          }
          if (i + 1 == cnt) break;
          sharma_step<DT>(S, B, st, C);
        }
      }
      // reverse the chunk's steps, one stage at a time (C, B, A)
#pragma unroll 1
      for (int i = KS - 1; i >= 0; --i) {
        const bool act = lane_chunk && (c0 + i < n);
        // the samples of stages A and B: their forces K1, K2 locate P2 and P3 (the same
        // arithmetic as the forward's), their derivatives serve the reverse of the stage
        SampleRev R1, R2, R3;
        Cell Q1;
        float wA[3], wB[3];
        if (act) {
          // recompute the step's three sample points (same arithmetic as the forward)
          State s;
          s.jf = (float)(2 * (c0 + i));
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            s.d[a] = replay[(i * 6 + a) * 64 + lane];
            s.e[a] = replay[(i * 6 + 3 + a) * 64 + lane];
            s.bh[a] = fmaf(s.jf, B.g2hi[a], B.U0hi[a]);
          }
          float bh[3], sm[3];
          locate_state(S, B, s, Q1);
          sample_rev<DT>(S, Q1, R1);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            bh[a] = s.bh[a] + B.g2hi[a];
            sm[a] = small_part(B, a, s.jf + 1.0f, stage2_dev(S, s, a, R1.eta * R1.g[a]));  // as force_code
          }
          Cell Q2;
          locate3(S, bh, sm, Q2);
          sample_rev<DT>(S, Q2, R2);
          Cell Q3;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            bh[a] = bh[a] + B.g2hi[a];
            sm[a] = small_part(B, a, s.jf + 2.0f, stage3_dev(S, a, stage3_base(S, s, a), R2.eta * R2.g[a]));
          }
          locate3(S, bh, sm, Q3);
          sample_rev<DT>(S, Q3, R3);
          stage_weights(S, rb, tb, wA, wB);
        }
        reverse_stages<PARK>(S, A, P, act, R1, R2, R3, wA, wB, rb, tb, lane);
      }
      chunk_end(S, P, lane);
    }
  }
  // v0 from the ray header again rather than held in registers through the sweep
  float V0[3] = {0.0f, 0.0f, 0.0f};
  if (active) {
#pragma unroll
    for (int a = 0; a < 3; ++a) V0[a] = gld(S.ckpt + (size_t)q + (size_t)(12 + a) * (size_t)S.ckpt_pad);
  }
  entry_term<PARK>(S, B, V0, active, tb, A, P, lane);
  drain(S, A, P, lane);
}

// Recording form (checkpoint strides KS = 3 and 4, one chunk per checkpoint segment): the
// replay of a chunk keeps, for each of its steps, the record index and fractions of the
// step's three samples as the forward located them (16 bytes per sample and lane in LDS, sample s of
// step i of lane l at [(i * 3 + s) * 64 + l]). The reverse of a step then reads them back,
// issues its three cell gathers together and evaluates value, gradient and mixed second
// derivatives at exactly the forward's cells and fractions, without relocating the
// samples from the state (no stage points, no K1 / K2, no dependent gathers).
template <int KS>
constexpr int rec_floats_per_wave() { return KS * 3 * 64 * 4 + PEND_SLOTS * 8; }

// Chunks between two write-outs of the cache's stale slots.
template <int KS>
constexpr int rec_writeout_chunks() { return KS == 3 ? 3 : 2; }

// Recorder of the replay: sample s of the step at row[s * 64].
struct SampleRow {
  f32x4* row;
  __device__ __forceinline__ void operator()(int stage, unsigned rec, const Cell& Cs) const {
    row[stage * 64] = f32x4{__uint_as_float(rec), Cs.f[0], Cs.f[1], Cs.f[2]};
  }
};

template <int DT, int KS>
__device__ __forceinline__ void adjoint_tile_rec(const SceneDev& S, int tile, int lane, float* __restrict__ lds) {
  constexpr bool PARK = rec_waves_per_simd<KS>() == 3;  // registers for the parks
  AdjRay R;
  adjoint_ray_setup(S, tile, lane, R);
  const int q = R.q, n = R.n;
  const bool active = R.active;
  const RayBase& B = R.B;
  float* rb = R.rb;
  float* tb = R.tb;
  // the launcher takes this form only for a checkpoint stride of KS: a segment is one chunk
  const int nseg = wave_max_nonneg(active ? (n + KS - 1) / KS : 0);

  Accum A;
  accum_init(A);
  Pending P{lds + KS * 3 * 64 * 4, CELL_NONE, 0, 0u, 0u};
  f32x4* smp = reinterpret_cast<f32x4*>(lds);

  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int c0 = seg * KS;  // first step of the chunk
    const bool lane_chunk = active && c0 < n;
    // Wave priority, lowest to highest: the replay (a chain of dependent gathers), the
    // reverse (independent gathers, long VALU runs), the merge (serial wavefront
    // reductions, raised in `enter`). Each ordering step measured -2 % adjoint time in
    // alternating runs, whatever the levels.
    __builtin_amdgcn_s_setprio(0);
    if (lane_chunk) {
      State st;
      Cell C;
      state_at_step(B, c0, st);
      if (seg == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) { st.d[a] = 0.0f; st.e[a] = 0.0f; }
      } else {
        load_ckpt(S, q, seg - 1, st);
      }
      locate_state(S, B, st, C);
      // the chunk's steps, the last one only up to its third sample
      const int cnt = min(KS, n - c0);
#pragma unroll 1
      for (int i = 0; i < cnt - 1; ++i) sharma_step<DT>(S, B, st, C, SampleRow{smp + i * 3 * 64 + lane});
      sharma_step<DT, SampleRow, NoIssue, false>(S, B, st, C, SampleRow{smp + (cnt - 1) * 3 * 64 + lane});
    }
    // reverse the chunk's steps, one stage at a time (C, B, A)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll  // one copy per step: 1 % faster than the rolled loop, same registers
    for (int i = KS - 1; i >= 0; --i) {
      const bool act = lane_chunk && (c0 + i < n);
      SampleRev R1, R2, R3;
      float wA[3], wB[3];
      if (act) {
        const f32x4* row = smp + i * 3 * 64 + lane;
        const f32x4 s1 = row[0], s2 = row[64], s3 = row[128];
        const unsigned r1 = __float_as_uint(s1.x), r2 = __float_as_uint(s2.x), r3 = __float_as_uint(s3.x);
        float c1[8], c2[8], c3[8];
        fetch_cell<DT>(S, r3, c3);
        fetch_cell<DT>(S, r2, c2);
        fetch_cell<DT>(S, r1, c1);
        const float f3[3] = {s3.y, s3.z, s3.w}, f2[3] = {s2.y, s2.z, s2.w}, f1[3] = {s1.y, s1.z, s1.w};
        sample_rev_at(S, c3, r3, f3, R3);
        sample_rev_at(S, c2, r2, f2, R2);
        sample_rev_at(S, c1, r1, f1, R1);
        stage_weights(S, rb, tb, wA, wB);
      }
      reverse_stages<PARK>(S, A, P, act, R1, R2, R3, wA, wB, rb, tb, lane);
    }
    // stale slots go out every ~8 steps: each write-out exposes its atomics' latency once,
    // and at every chunk of 3 steps that cost showed (-2 % adjoint time at 9 steps; at 12 or
    // more the cache fills and misses write slots out one at a time)
    if (seg % rec_writeout_chunks<KS>() == 0) chunk_end(S, P, lane);
  }
  float V0[3] = {0.0f, 0.0f, 0.0f};
  if (active) {
#pragma unroll
    for (int a = 0; a < 3; ++a) V0[a] = gld(S.ckpt + (size_t)q + (size_t)(12 + a) * (size_t)S.ckpt_pad);
  }
  entry_term<PARK>(S, B, V0, active, tb, A, P, lane);
  drain(S, A, P, lane);
}

template <int DT, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(rec_waves_per_simd<KS>()))) void k_trace_adj_rec(
    const SceneDev* __restrict__ scenes, int n_scenes, int total_tiles, int wpb, int nblocks) {
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int gtile = xcd_remap(blockIdx.x, nblocks) * wpb + wave;
  if (gtile >= total_tiles) return;  // whole wavefront
  const int si = find_scene(scenes, n_scenes, gtile);
  const SceneDev& S = scenes[si];
  extern __shared__ float lds[];
  adjoint_tile_rec<DT, KS>(S, gtile - S.tile_begin, lane, lds + wave * rec_floats_per_wave<KS>());
}

template <int DT, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(rec_waves_per_simd<KS>()))) void k_trace_adj_rec_persistent(
    const SceneDev* __restrict__ scenes, int n_scenes, int total_tiles, unsigned int* __restrict__ queues,
    const int* __restrict__ order) {
  const int lane = threadIdx.x & 63, wave = wave_uniform(threadIdx.x >> 6);
  const int xcd = blockIdx.x & 7;
  extern __shared__ float lds[];
  float* mine = lds + wave * rec_floats_per_wave<KS>();
  for (int q = 0; q < 8; ++q) {
    const int qx = (xcd + q) & 7;
    int q_begin, q_end;
    xcd_tile_range(total_tiles, qx, q_begin, q_end);
    while (true) {
      int t = 0;
      if (lane == 0) t = (int)atomicAdd(&queues[8 + qx], 1u);
      t = wave_uniform(t) + q_begin;  // lane 0's claim (all lanes active)
      if (t >= q_end) break;
      t = wave_uniform(gld(order + t));
      const int si = find_scene(scenes, n_scenes, t);
      const SceneDev& S = scenes[si];
      adjoint_tile_rec<DT, KS>(S, t - S.tile_begin, lane, mine);
    }
  }
}

template <int DT, int KS>
static hipError_t launch_adj_rec(const LaunchPlan& P, hipStream_t stream) {
  if (P.ckpt_k != KS) return hipErrorInvalidValue;  // one chunk per checkpoint segment
  const size_t lds = sizeof(float) * rec_floats_per_wave<KS>() * (size_t)P.wpb;
  if (P.persistent) {
    const int grid = persistent_grid(k_trace_adj_rec_persistent<DT, KS>, P, lds);
    hipLaunchKernelGGL((k_trace_adj_rec_persistent<DT, KS>), dim3(grid), dim3(64 * P.wpb), lds, stream, P.scenes,
                       P.n_scenes, P.total_tiles, P.queues, P.tile_order);
  } else {
    int nblocks = (P.total_tiles + P.wpb - 1) / P.wpb;
    hipLaunchKernelGGL((k_trace_adj_rec<DT, KS>), dim3(nblocks), dim3(64 * P.wpb), lds, stream, P.scenes,
                       P.n_scenes, P.total_tiles, P.wpb, nblocks);
  }
  return hipGetLastError();
}

// Quasi-linear form: the stage points lie on the entry line, at its half-step points
// j = 0 .. 2n (P(j) = U0 + j g2, g2 = V h / 2 in grid units), so the reverse needs no
// states. The state recursion is linear: with r = dL/dd and tau_k = dL/de after step k,
// r stays rb and tau_k = tb + (n - k) h rb. The force at P(j) gets the adjoint
//   even j = 2m: h (h/6 r + tau_{m+1}/6) [stage A of step m, m < n]
//                + h tau_m / 6 [stage C of step m - 1, m > 0]
//   odd  j = 2k + 1: h (h/3 r + 2/3 tau_{k+1}) [stage B of step k]
// and passes it to the 8 corner voxels and, through the point's dependence on the
// entry velocity, j h/2 times its position adjoint to dL/dv0.
template <int DT>
__device__ __forceinline__ void adjoint_tile_ql(const SceneDev& S, int tile, int lane, float* __restrict__ cache) {
  AdjRay R;
  adjoint_ray_setup(S, tile, lane, R);
  const int n = R.n;
  const bool active = R.active;
  const RayBase& B = R.B;
  const int npts = wave_max_nonneg(active ? 2 * n + 1 : 0);
  const float h = S.hf, h_6 = S.h_6;
  Accum A;
  accum_init(A);
  Pending P{cache, CELL_NONE, 0, 0u, 0u};
  float pv[3] = {0.0f, 0.0f, 0.0f};  // dL/dv0 through the stage points (grid units)
#pragma unroll 1
  for (int j = 0; j < npts; ++j) {
    const bool act = active && j <= 2 * n;
    SampleRev Rs;
    float w[3];
    if (act) {
      float v[3];
      const int m = j >> 1;
      if ((j & 1) == 0) {
        const float ca = (float)(n - m - 1) * h, cc = (float)(n - m) * h;  // tau_{m+1}, tau_m
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float tA = fmaf(ca, R.rb[a], R.tb[a]), tC = fmaf(cc, R.rb[a], R.tb[a]);
          const float wa = m < n ? h * fmaf(h_6, R.rb[a], tA * (1.0f / 6.0f)) : 0.0f;
          const float wc = m > 0 ? h * (tC * (1.0f / 6.0f)) : 0.0f;
          v[a] = wa + wc;
        }
      } else {
        const float cb = (float)(n - m - 1) * h;  // tau_{m+1}
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float tB = fmaf(cb, R.rb[a], R.tb[a]);
          v[a] = h * fmaf(h * (1.0f / 3.0f), R.rb[a], tB * (2.0f / 3.0f));
        }
      }
      const float jf = (float)j;
      float bh[3], sm[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bh[a] = fmaf(jf, B.g2hi[a], B.U0hi[a]);
        sm[a] = small_part(B, a, jf, 0.0f);
      }
      Cell C;
      locate3(S, bh, sm, C);
      sample_rev<DT>(S, C, Rs);
#pragma unroll
      for (int a = 0; a < 3; ++a) w[a] = v[a] * S.km[a];  // dL/dK -> dL/dG
    }
    enter<true>(S, A, act, __ballot(act), act ? Rs.key : 0, lane, P);
    if (act) {
      float p[3];
      force_rev(S, Rs, w, p, A.acc);
      const float tj = (float)j * (0.5f * h);
#pragma unroll
      for (int a = 0; a < 3; ++a) pv[a] = fmaf(tj, p[a], pv[a]);
    }
    if ((j & 15) == 15) chunk_end(S, P, lane);
  }
  float tb0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) tb0[a] = fmaf((float)n * h, R.rb[a], R.tb[a]) + pv[a];
  entry_term<true>(S, B, B.V, active, tb0, A, P, lane);
  drain(S, A, P, lane);
}

// Held to 80 registers for 6 wavefronts per SIMD: this latency-bound grid form runs 4 %
// faster that way, its small spill included (the persistent form gains nothing from it).
template <int DT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_trace_adj_ql(
    const SceneDev* __restrict__ scenes, int n_scenes, int total_tiles, int wpb, int nblocks) {
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int gtile = xcd_remap(blockIdx.x, nblocks) * wpb + wave;
  if (gtile >= total_tiles) return;  // whole wavefront
  const int si = find_scene(scenes, n_scenes, gtile);
  const SceneDev& S = scenes[si];
  extern __shared__ float lds[];
  adjoint_tile_ql<DT>(S, gtile - S.tile_begin, lane, lds + wave * (PEND_SLOTS * 8));
}

template <int DT>
__global__ __launch_bounds__(256) void k_trace_adj_ql_persistent(const SceneDev* __restrict__ scenes, int n_scenes,
                                                                 int total_tiles, unsigned int* __restrict__ queues,
                                                                 const int* __restrict__ order) {
  const int lane = threadIdx.x & 63, wave = wave_uniform(threadIdx.x >> 6);
  const int xcd = blockIdx.x & 7;
  extern __shared__ float lds[];
  float* cache = lds + wave * (PEND_SLOTS * 8);
  for (int q = 0; q < 8; ++q) {
    const int qx = (xcd + q) & 7;
    int q_begin, q_end;
    xcd_tile_range(total_tiles, qx, q_begin, q_end);
    while (true) {
      int t = 0;
      if (lane == 0) t = (int)atomicAdd(&queues[8 + qx], 1u);
      t = wave_uniform(t) + q_begin;  // lane 0's claim (all lanes active)
      if (t >= q_end) break;
      t = wave_uniform(gld(order + t));
      const int si = find_scene(scenes, n_scenes, t);
      const SceneDev& S = scenes[si];
      adjoint_tile_ql<DT>(S, t - S.tile_begin, lane, cache);
    }
  }
}

template <int DT>
static hipError_t launch_adj_ql(const LaunchPlan& P, hipStream_t stream) {
  const size_t lds = sizeof(float) * PEND_SLOTS * 8 * (size_t)P.wpb;
  if (P.persistent) {
    const int grid = persistent_grid(k_trace_adj_ql_persistent<DT>, P, lds);
    hipLaunchKernelGGL((k_trace_adj_ql_persistent<DT>), dim3(grid), dim3(64 * P.wpb), lds, stream, P.scenes,
                       P.n_scenes, P.total_tiles, P.queues, P.tile_order);
  } else {
    int nblocks = (P.total_tiles + P.wpb - 1) / P.wpb;
    hipLaunchKernelGGL((k_trace_adj_ql<DT>), dim3(nblocks), dim3(64 * P.wpb), lds, stream, P.scenes, P.n_scenes,
                       P.total_tiles, P.wpb, nblocks);
  }
  return hipGetLastError();
}

template <int DT, int KS, bool STORED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(adj_waves_per_simd<KS>()))) void k_trace_adj(
    const SceneDev* __restrict__ scenes, int n_scenes, int total_tiles, int wpb, int nblocks) {
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int gtile = xcd_remap(blockIdx.x, nblocks) * wpb + wave;
  if (gtile >= total_tiles) return;  // whole wavefront
  const int si = find_scene(scenes, n_scenes, gtile);
  const SceneDev& S = scenes[si];
  extern __shared__ float lds[];
  adjoint_tile<DT, KS, STORED>(S, gtile - S.tile_begin, lane, lds + wave * lds_floats_per_wave<KS>());
}

template <int DT, int KS, bool STORED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(adj_waves_per_simd<KS>()))) void k_trace_adj_persistent(
    const SceneDev* __restrict__ scenes, int n_scenes, int total_tiles, unsigned int* __restrict__ queues,
    const int* __restrict__ order) {
  const int lane = threadIdx.x & 63, wave = wave_uniform(threadIdx.x >> 6);
  const int xcd = blockIdx.x & 7;
  extern __shared__ float lds[];
  float* replay = lds + wave * lds_floats_per_wave<KS>();
  for (int q = 0; q < 8; ++q) {
    const int qx = (xcd + q) & 7;
    int q_begin, q_end;
    xcd_tile_range(total_tiles, qx, q_begin, q_end);
    while (true) {
      int t = 0;
      if (lane == 0) t = (int)atomicAdd(&queues[8 + qx], 1u);
      t = wave_uniform(t) + q_begin;  // lane 0's claim (all lanes active)
      if (t >= q_end) break;
      t = wave_uniform(gld(order + t));
      const int si = find_scene(scenes, n_scenes, t);
      const SceneDev& S = scenes[si];
      adjoint_tile<DT, KS, STORED>(S, t - S.tile_begin, lane, replay);
    }
  }
}

template <int DT, int KS, bool STORED>
static hipError_t launch_adj_t(const LaunchPlan& P, hipStream_t stream) {
  const size_t lds = sizeof(float) * lds_floats_per_wave<KS>() * (size_t)P.wpb;
  if (P.persistent) {
    const int grid = persistent_grid(k_trace_adj_persistent<DT, KS, STORED>, P, lds);
    hipLaunchKernelGGL((k_trace_adj_persistent<DT, KS, STORED>), dim3(grid), dim3(64 * P.wpb), lds, stream,
                       P.scenes, P.n_scenes, P.total_tiles, P.queues, P.tile_order);
  } else {
    int nblocks = (P.total_tiles + P.wpb - 1) / P.wpb;
    hipLaunchKernelGGL((k_trace_adj<DT, KS, STORED>), dim3(nblocks), dim3(64 * P.wpb), lds, stream, P.scenes,
                       P.n_scenes, P.total_tiles, P.wpb, nblocks);
  }
  return hipGetLastError();
}

template <int DT>
static hipError_t launch_adj_dt(const LaunchPlan& P, hipStream_t stream) {
  if (P.tracer == 1) return launch_adj_ql<DT>(P, stream);
  // chunks of step-start states in LDS: stride 1 fills chunks of 8 from the checkpoints,
  // stride 6 replays chunks of 6, strides 8, 16, ... chunks of 8
  if (P.ckpt_k == 1) return launch_adj_t<DT, 8, true>(P, stream);
  if (P.ckpt_k == 3) return launch_adj_rec<DT, 3>(P, stream);
  if (P.ckpt_k == 4) return launch_adj_rec<DT, 4>(P, stream);
  if (P.ckpt_k == 6) return launch_adj_t<DT, 6, false>(P, stream);
  return launch_adj_t<DT, 8, false>(P, stream);
}

// Processing order of the persistent adjoint. A tile's reverse sweep lasts as long as
// its longest ray, and the tiles of the per-XCD ranges differ by up to ~1.5x (rays that
// leave the box through a side face are short). Taken in index order, the long tiles
// that start last leave most wavefront slots idle at the end of the launch. Each range
// is therefore taken longest first: its tiles are counting-sorted by the forward's
// largest step count (ties in any order), so the short tiles fill the end.
__global__ __launch_bounds__(256) void k_tile_cost(const SceneDev* __restrict__ scenes, int n_scenes, int total_tiles,
                                                   int* __restrict__ cost) {
  const int wave = wave_uniform(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int gtile = blockIdx.x * 4 + wave;
  if (gtile >= total_tiles) return;  // whole wavefront
  const SceneDev& S = scenes[find_scene(scenes, n_scenes, gtile)];
  int r = 0, pix = 0, smp = 0, n = 0;
  if (tile_ray(S, gtile - S.tile_begin, lane, r, pix, smp)) n = max(gld(S.n_steps + r), 0);
  n = wave_max_nonneg(n);  // all 64 lanes active
  if (lane == 0) cost[gtile] = n;
}

constexpr int ORDER_KEYS = 1024;

__device__ __forceinline__ int order_key(int cost, int shift) {
  return ORDER_KEYS - 1 - min(cost >> shift, ORDER_KEYS - 1);  // longest first
}

// one block per XCD: the tiles it owns, longest first, into its range [b, e) of order
__global__ __launch_bounds__(ORDER_KEYS) void k_tile_order(const int* __restrict__ cost, int total_tiles, int shift,
                                                           int* __restrict__ order) {
  __shared__ int start[ORDER_KEYS];
  const int tid = threadIdx.x, x = blockIdx.x;
  int b, e;
  xcd_tile_range(total_tiles, x, b, e);
  start[tid] = 0;
  __syncthreads();
  for (int i = tid; i < e - b; i += ORDER_KEYS)
    atomicAdd(&start[order_key(gld(cost + xcd_tile(total_tiles, x, i)), shift)], 1);
  __syncthreads();
  // exclusive prefix sum of the key counts (Hillis-Steele)
  const int count = start[tid];
  int v = count;
  for (int d = 1; d < ORDER_KEYS; d <<= 1) {
    const int add = tid >= d ? start[tid - d] : 0;
    __syncthreads();
    v += add;
    start[tid] = v;
    __syncthreads();
  }
  start[tid] = v - count;
  __syncthreads();
  for (int i = tid; i < e - b; i += ORDER_KEYS) {
    const int t = xcd_tile(total_tiles, x, i);
    const int pos = atomicAdd(&start[order_key(gld(cost + t), shift)], 1);
    order[b + pos] = t;
  }
}

hipError_t launch_tile_order(const LaunchPlan& P, hipStream_t stream) {
  if (P.total_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_cost, dim3((P.total_tiles + 3) / 4), dim3(256), 0, stream, P.scenes, P.n_scenes,
                     P.total_tiles, P.tile_cost);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_order, dim3(8), dim3(ORDER_KEYS), 0, stream, P.tile_cost, P.total_tiles, P.order_shift,
                     P.tile_order);
  return hipGetLastError();
}

hipError_t launch_trace_adj(const LaunchPlan& P, hipStream_t stream) {
  if (P.total_tiles == 0) return hipSuccess;
  switch (P.dtype) {
    case DT_F32: return launch_adj_dt<DT_F32>(P, stream);
    case DT_F16: return launch_adj_dt<DT_F16>(P, stream);
    case DT_BF16: return launch_adj_dt<DT_BF16>(P, stream);
    case DT_F32_XPAIR: return launch_adj_dt<DT_F32_XPAIR>(P, stream);
    case DT_F16_XPAIR: return launch_adj_dt<DT_F16_XPAIR>(P, stream);
    default: return launch_adj_dt<DT_BF16_XPAIR>(P, stream);
  }
}

}  // namespace rbos
