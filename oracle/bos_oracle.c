/*
 * bos_oracle.c -- plain, slow, obviously-correct FP64 oracle for single-view BOS ray
 * tracing (Teh, Ali, Rapp, Mansour, "Indoor Airflow Imaging Using Physics-Informed
 * Background-Oriented Schlieren Tomography").
 *
 * TEST INFRASTRUCTURE ONLY. It shares no code with the GPU library.
 *
 * Contents, in the paper's order:
 *   Sec. 2.A  refractive index from temperature, eta = 1 + rho0 G T0 / T, and the
 *             storage codes of eta - 1.
 *   Sec. 2.B  Eq. (1): dx/dt = v, dv/dt = eta grad(eta) ("nonlinear ray tracing"),
 *             integrated with Sharma's three-stage Runge-Kutta-Nystrom scheme (the
 *             ODE's cited source) on a trilinearly interpolated, cell-centred voxel
 *             field; box-only integration, straight lines outside.
 *   Sec. 2.C  Eq. (2) with one ray per pixel centre and the luminance term only: the
 *             traced ray's back-wall hit is rendered as the printed texture or the
 *             pinhole-projector image (bilinear).
 *   Sec. 2.D  L_BOS = sum_j |I_flow^j - I^j(eta)|^2 and its exact gradient with respect
 *             to eta - 1 at every voxel: the discrete adjoint of the three steps above.
 *             A tangent-linear model and branch-locked central differences check it.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off, no fast-math. binary64 everywhere except
 * the binary32 arithmetic that decides stored codes.
 */
#include "bos_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

int or_version(void) { return 1; }
int or_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------------------ */
/* small vector helpers                                                                  */
/* ------------------------------------------------------------------------------------ */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void axpy3(double* y, double a, const double* x) { y[0] += a * x[0]; y[1] += a * x[1]; y[2] += a * x[2]; }
static void matvec3(double m[3][3], const double* x, double* y) {
  for (int i = 0; i < 3; ++i) y[i] = m[i][0] * x[0] + m[i][1] * x[1] + m[i][2] * x[2];
}
static int finite3(const double* a) { return isfinite(a[0]) && isfinite(a[1]) && isfinite(a[2]); }

/* ------------------------------------------------------------------------------------ */
/* Sec. 2.A: eta(T) and storage codes                                                    */
/* ------------------------------------------------------------------------------------ */
int or_delta_from_temperature(const float* T, int64_t n, double rho0G, double T0, double* delta) {
  if (!T || !delta || n < 0) return -1;
  for (int64_t i = 0; i < n; ++i) delta[i] = rho0G * T0 / (double)T[i];
  return 0;
}

int or_delta_from_temperature_f32(const float* T, int64_t n, float rho0G, float T0, float* delta) {
  if (!T || !delta || n < 0) return -1;
  for (int64_t i = 0; i < n; ++i) {
    volatile float ratio = T0 / T[i]; /* one binary32 rounding */
    delta[i] = rho0G * ratio;         /* a second binary32 rounding */
  }
  return 0;
}

/* Round a finite binary64 value to the nearest (ties to even) number with `mant` stored
   mantissa bits and exponent bias `bias`, and return its bit pattern (sign | exp | mant). */
static uint16_t round_to_small_float(double x, int mant, int bias) {
  uint16_t sign = signbit(x) ? (uint16_t)(1u << (mant + (mant == 10 ? 5 : 8))) : 0;
  int exp_bits = (mant == 10) ? 5 : 8;
  if (isnan(x)) return (uint16_t)(((1u << exp_bits) - 1u) << mant | (1u << (mant - 1)));
  double ax = fabs(x);
  if (ax == 0.0) return sign;
  int e2;
  frexp(ax, &e2);         /* ax in [2^(e2-1), 2^e2) */
  int E = e2 - 1;
  int emin = 1 - bias;    /* smallest normal exponent */
  if (E < emin) E = emin; /* subnormals share the quantum of the smallest binade */
  double quantum = ldexp(1.0, E - mant);
  double q = rint(ax / quantum); /* round to nearest, ties to even (default mode) */
  if (q >= ldexp(1.0, mant + 1)) { q *= 0.5; E += 1; } /* rounded up into the next binade */
  int emax = bias;
  if (E > emax) return (uint16_t)(sign | (((1u << exp_bits) - 1u) << mant)); /* infinity */
  if (q < ldexp(1.0, mant)) return (uint16_t)(sign | (uint16_t)q);           /* subnormal */
  return (uint16_t)(sign | (uint16_t)((unsigned)(E + bias) << mant) |
                    (uint16_t)(q - ldexp(1.0, mant)));
}

static double small_float_value(uint16_t bits, int mant, int bias) {
  int exp_bits = (mant == 10) ? 5 : 8;
  int sign = (bits >> (mant + exp_bits)) & 1;
  int e = (bits >> mant) & ((1 << exp_bits) - 1);
  int m = bits & ((1 << mant) - 1);
  double v;
  if (e == 0) v = ldexp((double)m, 1 - bias - mant);
  else if (e == (1 << exp_bits) - 1) v = m ? NAN : INFINITY;
  else v = ldexp((double)(m + (1 << mant)), e - bias - mant);
  return sign ? -v : v;
}

int or_encode(const float* delta, int64_t n, int32_t code, double scale, double offset, void* codes) {
  if (!delta || !codes || n < 0 || !(scale > 0.0)) return -1;
  float c = (float)offset, s = (float)scale;
  for (int64_t i = 0; i < n; ++i) {
    volatile float t = delta[i] - c; /* binary32 */
    volatile float q = t * s;        /* binary32 (exact for a power-of-two scale) */
    if (code == OR_CODE_F32) ((float*)codes)[i] = q;
    else if (code == OR_CODE_F16) ((uint16_t*)codes)[i] = round_to_small_float((double)q, 10, 15);
    else if (code == OR_CODE_BF16) ((uint16_t*)codes)[i] = round_to_small_float((double)q, 7, 127);
    else return -2;
  }
  return 0;
}

int or_decode(const void* codes, int64_t n, int32_t code, double scale, double offset, double* delta) {
  if (!delta || !codes || n < 0 || !(scale > 0.0)) return -1;
  double c = (double)(float)offset;
  for (int64_t i = 0; i < n; ++i) {
    double q;
    if (code == OR_CODE_F32) q = (double)((const float*)codes)[i];
    else if (code == OR_CODE_F16) q = small_float_value(((const uint16_t*)codes)[i], 10, 15);
    else if (code == OR_CODE_BF16) q = small_float_value(((const uint16_t*)codes)[i], 7, 127);
    else return -2;
    delta[i] = c + q / scale;
  }
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* The field: eta - 1 and its derivatives at a point                                     */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  int32_t i0[3];      /* lower corner voxel per axis */
  int32_t clamped[3]; /* axis outside the voxel-centre range (field held constant) */
  double fcl[3];      /* fraction used on a clamped axis (0 or 1) */
} cell_t;

typedef struct {
  double delta, grad[3], hess[3][3];
  /* grid mode: cell, per-axis weights w[a][0] = 1 - f, w[a][1] = f and their
     derivatives dw[a][k] = d w[a][k] / d x_a (zero on a clamped axis) */
  cell_t cell;
  double w[3][2], dw[3][2];
} sample_t;

static double field_voxel(const or_field* F, int i, int j, int k) {
  int64_t idx = ((int64_t)k * F->n[1] + j) * F->n[0] + i;
  double v = F->delta[idx];
  if (idx == F->pert_index) v += F->pert_value;
  return v;
}

/* Trilinear interpolation over cell-centred voxels, clamp-to-edge; the gradient and
   Hessian are those of the interpolant. Along each axis the interpolation cell of u is
   [i, i+1) with i = floor(u); u < 0 and u >= n - 1 are outside the centres, where the
   field is held at the edge values (zero derivative along that axis). lock != NULL reuses a recorded cell (and the
   clamp decisions) instead of locating P. */
static void sample_grid(const or_field* F, const double* P, const cell_t* lock, sample_t* s) {
  for (int a = 0; a < 3; ++a) {
    int n = F->n[a];
    double dx = (F->hi[a] - F->lo[a]) / n;
    double u = (P[a] - F->lo[a]) / dx - 0.5;
    int i0, cl;
    double f;
    if (lock) {
      i0 = lock->i0[a];
      cl = lock->clamped[a];
      f = cl ? lock->fcl[a] : u - i0;
    } else if (!(u >= 0.0)) { /* below the first centre, or not a number */
      i0 = 0; f = 0.0; cl = 1;
    } else if (u >= n - 1) { /* at or beyond the last centre: cells are half-open [i, i+1) */
      i0 = n - 2; f = 1.0; cl = 1;
    } else {
      i0 = (int)floor(u);
      f = u - i0; cl = 0;
    }
    s->cell.i0[a] = i0;
    s->cell.clamped[a] = cl;
    s->cell.fcl[a] = cl ? f : 0.0;
    s->w[a][0] = 1.0 - f;
    s->w[a][1] = f;
    s->dw[a][0] = cl ? 0.0 : -1.0 / dx;
    s->dw[a][1] = cl ? 0.0 : 1.0 / dx;
  }
  s->delta = 0.0;
  memset(s->grad, 0, sizeof s->grad);
  memset(s->hess, 0, sizeof s->hess);
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        double v = field_voxel(F, s->cell.i0[0] + a, s->cell.i0[1] + b, s->cell.i0[2] + c);
        double wx = s->w[0][a], wy = s->w[1][b], wz = s->w[2][c];
        double gx = s->dw[0][a], gy = s->dw[1][b], gz = s->dw[2][c];
        s->delta += wx * wy * wz * v;
        s->grad[0] += gx * wy * wz * v;
        s->grad[1] += wx * gy * wz * v;
        s->grad[2] += wx * wy * gz * v;
        s->hess[0][1] += gx * gy * wz * v;
        s->hess[0][2] += gx * wy * gz * v;
        s->hess[1][2] += wx * gy * gz * v;
      }
  s->hess[1][0] = s->hess[0][1];
  s->hess[2][0] = s->hess[0][2];
  s->hess[2][1] = s->hess[1][2];
}

static void sample_analytic(const or_field* F, const double* P, sample_t* s) {
  memset(s, 0, sizeof *s);
  double r[3] = {P[0] - F->c[0], P[1] - F->c[1], P[2] - F->c[2]};
  switch (F->mode) {
    case OR_FIELD_HOMOGENEOUS:
      s->delta = F->a;
      break;
    case OR_FIELD_LINEAR:
      s->delta = F->a + dot3(F->g, r);
      for (int i = 0; i < 3; ++i) s->grad[i] = F->g[i];
      break;
    case OR_FIELD_ETA2_LINEAR: {
      double eta = sqrt(F->a + dot3(F->g, r));
      s->delta = eta - 1.0;
      for (int i = 0; i < 3; ++i) s->grad[i] = F->g[i] / (2.0 * eta);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s->hess[i][j] = -F->g[i] * F->g[j] / (4.0 * eta * eta * eta);
      break;
    }
    case OR_FIELD_GAUSSIAN: {
      double s2 = F->sigma * F->sigma;
      double e = F->eps * exp(-dot3(r, r) / (2.0 * s2));
      s->delta = F->a + e;
      for (int i = 0; i < 3; ++i) s->grad[i] = -r[i] / s2 * e;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s->hess[i][j] = e * (r[i] * r[j] / (s2 * s2) - (i == j ? 1.0 / s2 : 0.0));
      break;
    }
  }
}

static void sample_field(const or_field* F, const double* P, const cell_t* lock, sample_t* s) {
  if (F->mode == OR_FIELD_GRID) sample_grid(F, P, lock, s);
  else sample_analytic(F, P, s);
}

/* Right-hand side of the velocity equation in Eq. (1): D = eta grad(eta) = (1 + delta) grad(delta). */
static void force(const sample_t* s, double* D) {
  double eta = 1.0 + s->delta;
  for (int i = 0; i < 3; ++i) D[i] = eta * s->grad[i];
}

/* J = dD/dx = grad(delta) grad(delta)^T + (1 + delta) Hess(delta), symmetric. */
static void force_jacobian(const sample_t* s, double J[3][3]) {
  double eta = 1.0 + s->delta;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) J[i][j] = s->grad[i] * s->grad[j] + eta * s->hess[i][j];
}

int or_sample(const or_field* F, const double* P, double* delta, double* grad, double* hess) {
  if (!F || !P) return -1;
  if (F->mode == OR_FIELD_GRID && (!F->delta || F->n[0] < 2 || F->n[1] < 2 || F->n[2] < 2)) return -1;
  sample_t s;
  sample_field(F, P, NULL, &s);
  if (delta) *delta = s.delta;
  if (grad) memcpy(grad, s.grad, sizeof s.grad);
  if (hess) memcpy(hess, s.hess, sizeof s.hess);
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Sec. 2.B: Eq. (1) with Sharma's scheme                                                */
/* ------------------------------------------------------------------------------------ */
/* One step of size h for x'' = D(x), with (x, v) the position and velocity of Eq. (1):
     A = h D(x)
     B = h D(x + h/2 v + h/8 A)
     C = h D(x + h v + h/2 B)
     x <- x + h (v + (A + 2B)/6),  v <- v + (A + 4B + C)/6.
   locks (nullable) receive / supply the cells of the three samples. */
typedef struct {
  double P[3][3];   /* stage points */
  sample_t s[3];    /* stage samples */
  double K[3][3];   /* A, B, C */
} stages_t;

static void sharma_step(const or_field* F, double h, const double* x, const double* v,
                        cell_t* locks, int use_locks, double* x_new, double* v_new, stages_t* st) {
  stages_t local;
  if (!st) st = &local;
  double D[3];
  for (int i = 0; i < 3; ++i) st->P[0][i] = x[i];
  sample_field(F, st->P[0], use_locks ? &locks[0] : NULL, &st->s[0]);
  force(&st->s[0], D);
  for (int i = 0; i < 3; ++i) st->K[0][i] = h * D[i];
  for (int i = 0; i < 3; ++i) st->P[1][i] = x[i] + 0.5 * h * v[i] + 0.125 * h * st->K[0][i];
  sample_field(F, st->P[1], use_locks ? &locks[1] : NULL, &st->s[1]);
  force(&st->s[1], D);
  for (int i = 0; i < 3; ++i) st->K[1][i] = h * D[i];
  for (int i = 0; i < 3; ++i) st->P[2][i] = x[i] + h * v[i] + 0.5 * h * st->K[1][i];
  sample_field(F, st->P[2], use_locks ? &locks[2] : NULL, &st->s[2]);
  force(&st->s[2], D);
  for (int i = 0; i < 3; ++i) st->K[2][i] = h * D[i];
  for (int i = 0; i < 3; ++i) {
    x_new[i] = x[i] + h * (v[i] + (st->K[0][i] + 2.0 * st->K[1][i]) / 6.0);
    v_new[i] = v[i] + (st->K[0][i] + 4.0 * st->K[1][i] + st->K[2][i]) / 6.0;
  }
  if (locks && !use_locks)
    for (int k = 0; k < 3; ++k) locks[k] = st->s[k].cell;
}

/* Quasi-linear form (Sec. 2.B): the path is approximated by the straight line
   L(t) = x0 + v0 t from the entry state; the field is queried on L to give the
   approximate velocity, which then drives the position. The same update as above, with
   the force taken on L at the stage times:
     A = h D(L(t)),  B = h D(L(t + h/2)),  C = h D(L(t + h)),
     x <- x + h (v + (A + 2B)/6),  v <- v + (A + 4B + C)/6.
   (With the force a function of t alone, the update is Simpson's rule for v and exact
   for cubic forcing.) */
static void quasi_step(const or_field* F, double h, const double* x0, const double* v0, double t,
                       const double* x, const double* v, cell_t* locks, int use_locks, double* x_new,
                       double* v_new, stages_t* st) {
  stages_t local;
  if (!st) st = &local;
  const double ts[3] = {t, t + 0.5 * h, t + h};
  double D[3];
  for (int k = 0; k < 3; ++k) {
    for (int i = 0; i < 3; ++i) st->P[k][i] = x0[i] + ts[k] * v0[i];
    sample_field(F, st->P[k], use_locks ? &locks[k] : NULL, &st->s[k]);
    force(&st->s[k], D);
    for (int i = 0; i < 3; ++i) st->K[k][i] = h * D[i];
  }
  for (int i = 0; i < 3; ++i) {
    x_new[i] = x[i] + h * (v[i] + (st->K[0][i] + 2.0 * st->K[1][i]) / 6.0);
    v_new[i] = v[i] + (st->K[0][i] + 4.0 * st->K[1][i] + st->K[2][i]) / 6.0;
  }
  if (locks && !use_locks)
    for (int k = 0; k < 3; ++k) locks[k] = st->s[k].cell;
}

/* Step n of a ray that entered at (x0, v0), in the scene's tracer form. */
static void ray_step(const or_field* F, const or_scene* S, const double* x0, const double* v0, int n,
                     const double* x, const double* v, cell_t* locks, int use_locks, double* x_new,
                     double* v_new, stages_t* st) {
  if (S->tracer == OR_TRACER_QUASILINEAR)
    quasi_step(F, S->step, x0, v0, n * S->step, x, v, locks, use_locks, x_new, v_new, st);
  else
    sharma_step(F, S->step, x, v, locks, use_locks, x_new, v_new, st);
}

int or_integrate_quasi(const or_field* F, const double* x0, const double* v0, double h, int32_t nsteps,
                       double* x_out, double* v_out) {
  if (!F || !x0 || !v0 || !x_out || !v_out || nsteps < 0) return -1;
  double x[3], v[3], xn[3], vn[3];
  memcpy(x, x0, sizeof x);
  memcpy(v, v0, sizeof v);
  for (int n = 0; n < nsteps; ++n) {
    quasi_step(F, h, x0, v0, n * h, x, v, NULL, 0, xn, vn, NULL);
    memcpy(x, xn, sizeof x);
    memcpy(v, vn, sizeof v);
  }
  memcpy(x_out, x, sizeof x);
  memcpy(v_out, v, sizeof v);
  return 0;
}

int or_integrate(const or_field* F, const double* x0, const double* v0, double h, int32_t nsteps,
                 double* x_out, double* v_out) {
  if (!F || !x0 || !v0 || !x_out || !v_out || nsteps < 0) return -1;
  double x[3], v[3], xn[3], vn[3];
  memcpy(x, x0, sizeof x);
  memcpy(v, v0, sizeof v);
  for (int n = 0; n < nsteps; ++n) {
    sharma_step(F, h, x, v, NULL, 0, xn, vn, NULL);
    memcpy(x, xn, sizeof x);
    memcpy(v, vn, sizeof v);
  }
  memcpy(x_out, x, sizeof x);
  memcpy(v_out, v, sizeof v);
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Sec. 2.C: camera, box, wall, wall luminance                                           */
/* ------------------------------------------------------------------------------------ */
/* Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as
   1, 2, 3", SC'11): ten rounds, each two 32 x 32 -> 64-bit products of the even counter
   words with fixed multipliers, the high halves mixed into the odd words with the key;
   the key advances by a Weyl sequence between rounds. */
static void philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

int or_philox4x32(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  if (!ctr || !key || !out) return -1;
  philox4x32_10(ctr, key, out);
  return 0;
}

/* Inverse CDF of the triangular density 1 - |x| on [-1, 1]. */
static double tent_inverse(double u) { return u < 0.5 ? sqrt(2.0 * u) - 1.0 : 1.0 - sqrt(2.0 - 2.0 * u); }

static void sample_offset(uint32_t seed, int32_t pixel, int32_t sample, double* ox, double* oy) {
  const uint32_t ctr[4] = {(uint32_t)pixel, (uint32_t)sample, 0u, 0u}, key[2] = {seed, 0u};
  uint32_t x[4];
  philox4x32_10(ctr, key, x);
  *ox = tent_inverse((double)(x[0] >> 8) * 0x1p-24);
  *oy = tent_inverse((double)(x[1] >> 8) * 0x1p-24);
}

int or_sample_offset(uint32_t seed, int32_t pixel, int32_t sample, double* ox, double* oy) {
  if (!ox || !oy || pixel < 0 || sample < 0) return -1;
  sample_offset(seed, pixel, sample, ox, oy);
  return 0;
}

/* Pinhole camera, horizontal field of view. With one sample per pixel the ray goes
   through the pixel centre; with more, through the centre plus the sample's offset
   (Eq. (2): the triangular camera filter, sampled by inverting its CDF). */
static void camera_ray(const or_scene* S, int32_t pix, int32_t sample, double* org, double* dir) {
  int col = pix % S->width, row = pix / S->width;
  double ox = 0.0, oy = 0.0;
  if (S->spp > 1) sample_offset(S->seed, pix, sample, &ox, &oy);
  double t = tan(0.5 * S->fov_x_deg * OR_PI / 180.0);
  double px = (2.0 * (col + 0.5 + ox) / S->width - 1.0) * t;
  double py = (1.0 - 2.0 * (row + 0.5 + oy) / S->height) * t * S->height / S->width;
  for (int i = 0; i < 3; ++i) {
    org[i] = S->cam_pos[i];
    dir[i] = S->cam_fwd[i] + px * S->cam_right[i] + py * S->cam_up[i];
  }
  double len = sqrt(dot3(dir, dir));
  for (int i = 0; i < 3; ++i) dir[i] /= len;
}

int or_camera_ray(const or_scene* S, int32_t pixel, double* org, double* dir) {
  if (!S || !org || !dir || pixel < 0 || pixel >= S->width * S->height) return -1;
  camera_ray(S, pixel, 0, org, dir);
  return 0;
}

/* Slab test; returns 1 with [t_in, t_out] when the line meets the box ahead of org. */
static int box_interval(const double* lo, const double* hi, const double* org, const double* dir,
                        double* t_in, double* t_out) {
  double tn = -INFINITY, tf = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (dir[a] != 0.0) {
      double t1 = (lo[a] - org[a]) / dir[a], t2 = (hi[a] - org[a]) / dir[a];
      double tmin = t1 < t2 ? t1 : t2, tmax = t1 < t2 ? t2 : t1;
      if (tmin > tn) tn = tmin;
      if (tmax < tf) tf = tmax;
    } else if (org[a] < lo[a] || org[a] > hi[a]) {
      return 0;
    }
  }
  double start = tn > 0.0 ? tn : 0.0;
  if (!(tf > start)) return 0;
  *t_in = start;
  *t_out = tf;
  return 1;
}

static int outside_box(const or_field* F, const double* x) {
  for (int a = 0; a < 3; ++a)
    if (x[a] < F->lo[a] || x[a] > F->hi[a]) return 1;
  return 0;
}

/* Straight transport to the back-wall plane: X = x + s v, s = ((p_w - x).n)/(v.n). */
static int wall_hit(const or_scene* S, const double* x, const double* v, double* X, double* s_out) {
  double vn = dot3(v, S->wall_normal);
  if (!(vn < 0.0)) return 0;
  double d[3] = {S->wall_origin[0] - x[0], S->wall_origin[1] - x[1], S->wall_origin[2] - x[2]};
  double s = dot3(d, S->wall_normal) / vn;
  for (int i = 0; i < 3; ++i) X[i] = x[i] + s * v[i];
  if (s_out) *s_out = s;
  return 1;
}

static void wall_coords(const or_scene* S, const double* X, double* uv) {
  double r[3] = {X[0] - S->wall_origin[0], X[1] - S->wall_origin[1], X[2] - S->wall_origin[2]};
  uv[0] = dot3(r, S->wall_u);
  uv[1] = dot3(r, S->wall_v);
}

/* Bilinear lookup with zero padding at texel coordinates (a, b) (column, row; texel
   centres at integers). tex (in/out) holds the lower texel (a0, b0); lock reuses it. */
static double bilinear(const double* img, int w, int h, double a, double b, int* tex, int lock,
                       double* dIda, double* dIdb, int* off) {
  int a0, b0;
  if (!lock && !(isfinite(a) && isfinite(b))) {
    *off = 1; *dIda = *dIdb = 0.0; tex[0] = tex[1] = 0;
    return 0.0;
  }
  if (lock) { a0 = tex[0]; b0 = tex[1]; }
  else { a0 = (int)floor(a); b0 = (int)floor(b); tex[0] = a0; tex[1] = b0; }
  double fa = a - a0, fb = b - b0;
  double t[2][2];
  int inside = 0;
  for (int j = 0; j < 2; ++j)
    for (int i = 0; i < 2; ++i) {
      int r = b0 + j, c = a0 + i;
      if (r >= 0 && r < h && c >= 0 && c < w) { t[j][i] = img[(int64_t)r * w + c]; inside = 1; }
      else t[j][i] = 0.0;
    }
  *off = !inside;
  *dIda = (1.0 - fb) * (t[0][1] - t[0][0]) + fb * (t[1][1] - t[1][0]);
  *dIdb = (1.0 - fa) * (t[1][0] - t[0][0]) + fa * (t[1][1] - t[0][1]);
  return (1.0 - fb) * ((1.0 - fa) * t[0][0] + fa * t[0][1]) + fb * ((1.0 - fa) * t[1][0] + fa * t[1][1]);
}

/* Luminance of the back wall at wall coordinates (u, v) and its (u, v) derivative.
   Printed: the texture spans [-E_u/2, E_u/2] x [-E_v/2, E_v/2] about the wall origin.
   Projector: a pinhole projector; the wall point is lit by the single projector pixel
   on its straight line to the projector centre; radiance = image value. */
static double wall_luminance(const or_scene* S, const double* uv, int* tex, int lock, double* dI, int* off) {
  double dIda, dIdb;
  if (S->wall_mode == OR_WALL_PRINTED) {
    double tu = S->pat_extent_u / S->pat_w, tv = S->pat_extent_v / S->pat_h;
    double a = (uv[0] + 0.5 * S->pat_extent_u) / tu - 0.5;
    double b = (0.5 * S->pat_extent_v - uv[1]) / tv - 0.5;
    double I = bilinear(S->pattern, S->pat_w, S->pat_h, a, b, tex, lock, &dIda, &dIdb, off);
    dI[0] = dIda / tu;
    dI[1] = -dIdb / tv;
    return I;
  }
  double X[3], Y[3];
  for (int i = 0; i < 3; ++i) X[i] = S->wall_origin[i] + uv[0] * S->wall_u[i] + uv[1] * S->wall_v[i];
  for (int i = 0; i < 3; ++i) Y[i] = X[i] - S->proj_pos[i];
  double z = dot3(Y, S->proj_fwd);
  if (!(z > 0.0)) { dI[0] = dI[1] = 0.0; *off = 1; return 0.0; }
  double tp = tan(0.5 * S->proj_fov_x_deg * OR_PI / 180.0);
  double sy = tp * (double)S->pat_h / (double)S->pat_w;
  double yr = dot3(Y, S->proj_right), yu = dot3(Y, S->proj_up);
  double xp = yr / (z * tp), yp = yu / (z * sy);
  double a = (xp + 1.0) * 0.5 * S->pat_w - 0.5;
  double b = (1.0 - yp) * 0.5 * S->pat_h - 0.5;
  double I = bilinear(S->pattern, S->pat_w, S->pat_h, a, b, tex, lock, &dIda, &dIdb, off);
  double dIdY[3];
  for (int i = 0; i < 3; ++i) {
    double dxp = S->proj_right[i] / (z * tp) - yr * S->proj_fwd[i] / (z * z * tp);
    double dyp = S->proj_up[i] / (z * sy) - yu * S->proj_fwd[i] / (z * z * sy);
    dIdY[i] = dIda * 0.5 * S->pat_w * dxp - dIdb * 0.5 * S->pat_h * dyp;
  }
  dI[0] = dot3(dIdY, S->wall_u);
  dI[1] = dot3(dIdY, S->wall_v);
  return I;
}

/* ------------------------------------------------------------------------------------ */
/* One ray: camera -> box -> Sharma steps -> wall                                        */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  int cap;          /* max steps */
  double* x;        /* states x_n, n = 0..n_steps, [cap+1][3] */
  double* v;
  cell_t* cells;    /* entry sample, then three stage samples per step */
  int n_steps;
  int entered;
  double org[3], dir[3], x0[3];
  int tex[2];
} tape_t;

static int tape_init(tape_t* t, int cap) {
  memset(t, 0, sizeof *t);
  t->cap = cap;
  t->x = (double*)malloc(sizeof(double) * 3 * (size_t)(cap + 1));
  t->v = (double*)malloc(sizeof(double) * 3 * (size_t)(cap + 1));
  t->cells = (cell_t*)malloc(sizeof(cell_t) * (size_t)(1 + 3 * cap));
  return t->x && t->v && t->cells;
}
static void tape_free(tape_t* t) { free(t->x); free(t->v); free(t->cells); }

typedef struct {
  double uv[2], uv0[2];
  int32_t n_steps;
  uint8_t status;
  double x[3], v[3];   /* last integrated state (straight camera ray when missed) */
  double path;         /* length of the ray path from the camera centre to the wall hit */
} ray_result_t;

static double dist3(const double* a, const double* b) {
  double d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  return sqrt(dot3(d, d));
}

/* unit vector from a to b */
static void unit_from_to(const double* a, const double* b, double* u) {
  double d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  double len = sqrt(dot3(d, d));
  for (int i = 0; i < 3; ++i) u[i] = d[i] / len;
}

/* Trace one ray. With locked != 0 the tape's cells and step count are replayed. */
static void trace_ray(const or_field* F, const or_scene* S, int32_t pix, int32_t sample, tape_t* tp, int locked,
                      ray_result_t* out) {
  double org[3], dir[3];
  camera_ray(S, pix, sample, org, dir);
  out->status = 0;
  out->n_steps = 0;
  out->path = NAN;
  double path = 0.0; /* polyline through the camera centre, the box entry and every state */
  double X[3];
  out->uv0[0] = out->uv0[1] = NAN;
  if (wall_hit(S, org, dir, X, NULL)) wall_coords(S, X, out->uv0);
  double t_in, t_out;
  int entered = box_interval(F->lo, F->hi, org, dir, &t_in, &t_out);
  if (tp) { memcpy(tp->org, org, sizeof org); memcpy(tp->dir, dir, sizeof dir); tp->entered = entered; }
  double x[3], v[3];
  if (!entered) {
    out->status |= OR_RAY_MISSED_BOX;
    memcpy(x, org, sizeof x);
    memcpy(v, dir, sizeof v);
  } else {
    /* Entry point and Sharma's initial condition |v| = eta. */
    for (int i = 0; i < 3; ++i) x[i] = org[i] + t_in * dir[i];
    sample_t s0;
    sample_field(F, x, (tp && locked) ? &tp->cells[0] : NULL, &s0);
    if (tp && !locked) tp->cells[0] = s0.cell;
    for (int i = 0; i < 3; ++i) v[i] = (1.0 + s0.delta) * dir[i];
    if (tp) { memcpy(tp->x0, x, sizeof x); memcpy(&tp->x[0], x, sizeof x); memcpy(&tp->v[0], v, sizeof v); }
    path = dist3(org, x);
    double x_in[3], v_in[3];
    memcpy(x_in, x, sizeof x);
    memcpy(v_in, v, sizeof v);
    int n_run = locked ? tp->n_steps : S->max_steps;
    int n = 0;
    for (; n < n_run; ++n) {
      double xn[3], vn[3];
      cell_t* lk = tp ? &tp->cells[1 + 3 * n] : NULL;
      ray_step(F, S, x_in, v_in, n, x, v, lk, locked, xn, vn, NULL);
      path += dist3(x, xn);
      memcpy(x, xn, sizeof x);
      memcpy(v, vn, sizeof v);
      if (tp) { memcpy(&tp->x[3 * (n + 1)], x, sizeof x); memcpy(&tp->v[3 * (n + 1)], v, sizeof v); }
      if (locked) continue;
      if (!finite3(x) || !finite3(v)) { out->status |= OR_RAY_NONFINITE; ++n; break; }
      if (outside_box(F, x)) { ++n; break; }
    }
    if (!locked && n == S->max_steps && !outside_box(F, x) && !(out->status & OR_RAY_NONFINITE))
      out->status |= OR_RAY_TRUNCATED;
    out->n_steps = n;
    if (tp && !locked) tp->n_steps = n;
  }
  memcpy(out->x, x, sizeof x);
  memcpy(out->v, v, sizeof v);
  if (out->status & OR_RAY_NONFINITE) { out->uv[0] = out->uv[1] = NAN; return; }
  double s_w;
  if (!wall_hit(S, x, v, X, &s_w)) {
    out->status |= OR_RAY_NO_WALL_HIT;
    out->uv[0] = out->uv[1] = NAN;
    return;
  }
  wall_coords(S, X, out->uv);
  /* the straight continuation to the wall, signed: negative when the last step ended
     past the wall plane (the wall on the box face), which takes the overshoot back */
  out->path = path + s_w * sqrt(dot3(v, v));
}

static int check_args(const or_field* F, const or_scene* S, const int32_t* ids, int32_t n_rays) {
  if (!F || !S || n_rays < 0 || S->spp < 1 || n_rays % S->spp) return -1;
  if (F->mode == OR_FIELD_GRID && (!F->delta || F->n[0] < 2 || F->n[1] < 2 || F->n[2] < 2)) return -1;
  if (S->width < 1 || S->height < 1 || !(S->step > 0.0) || S->max_steps < 1) return -1;
  if (!ids && n_rays != S->width * S->height * S->spp) return -1;
  return 0;
}

/* Ray r of n_rays is sample r / P of pixel index r % P (P = n_rays / spp pixels). */
static void ray_pixel(const or_scene* S, const int32_t* ids, int32_t n_rays, int32_t r, int32_t* pix,
                      int32_t* sample) {
  int32_t P = n_rays / S->spp, i = r % P;
  *sample = r / P;
  *pix = ids ? ids[i] : i;
}

int or_trace(const or_field* F, const or_scene* S, const int32_t* pixel_ids, int32_t n_rays,
             double* uv, double* duv, int32_t* n_steps, uint8_t* status, double* exit_xv, double* vdir,
             double* path) {
  if (check_args(F, S, pixel_ids, n_rays)) return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t r = 0; r < n_rays; ++r) {
    int32_t pix, sample;
    ray_pixel(S, pixel_ids, n_rays, r, &pix, &sample);
    ray_result_t res;
    trace_ray(F, S, pix, sample, NULL, 0, &res);
    if (vdir) {
      double len = sqrt(dot3(res.v, res.v));
      for (int i = 0; i < 3; ++i) vdir[3 * r + i] = res.v[i] / len;
    }
    if (path) path[r] = res.path;
    if (uv) { uv[2 * r] = res.uv[0]; uv[2 * r + 1] = res.uv[1]; }
    if (duv) { duv[2 * r] = res.uv[0] - res.uv0[0]; duv[2 * r + 1] = res.uv[1] - res.uv0[1]; }
    if (n_steps) n_steps[r] = res.n_steps;
    if (status) status[r] = res.status;
    if (exit_xv) { memcpy(&exit_xv[6 * r], res.x, 3 * sizeof(double)); memcpy(&exit_xv[6 * r + 3], res.v, 3 * sizeof(double)); }
  }
  return 0;
}

int or_render(const or_scene* S, const int32_t* pixel_ids, int32_t n_rays, const double* uv,
              uint8_t* status, double* image, double* dI_duv) {
  (void)pixel_ids;
  if (!S || !uv || !image || n_rays < 0 || !S->pattern || S->pat_w < 1 || S->pat_h < 1) return -1;
#pragma omp parallel for schedule(static)
  for (int32_t r = 0; r < n_rays; ++r) {
    double dI[2] = {0.0, 0.0};
    double I = 0.0;
    uint8_t st = status ? status[r] : 0;
    if (!(st & (OR_RAY_NO_WALL_HIT | OR_RAY_NONFINITE))) {
      int tex[2], off = 0;
      I = wall_luminance(S, &uv[2 * r], tex, 0, dI, &off);
      if (off && status) status[r] |= OR_RAY_OFF_PATTERN;
    }
    image[r] = I;
    if (dI_duv) { dI_duv[2 * r] = dI[0]; dI_duv[2 * r + 1] = dI[1]; }
  }
  return 0;
}

int or_loss(const double* image, const double* target, const double* dI_duv, int32_t n,
            double* loss, double* dL_duv) {
  if (!image || !target || n < 0) return -1;
  double L = 0.0;
  for (int32_t r = 0; r < n; ++r) {
    double res = image[r] - target[r];
    L += res * res;
    if (dL_duv && dI_duv) {
      dL_duv[2 * r] = 2.0 * res * dI_duv[2 * r];
      dL_duv[2 * r + 1] = 2.0 * res * dI_duv[2 * r + 1];
    }
  }
  if (loss) *loss = L;
  return 0;
}

/* Eq. (2) weight of a ray reaching the wall with unit direction d after a path of length
   ell: w = |<n_w, d>| / ell (the cosine between the wall normal and the direction, over
   the length of the ray path), and its derivatives w.r.t. d and ell. */
static double radiometric(const or_scene* S, const double* d, double ell, double* dw_dd, double* dw_dell) {
  double c = dot3(S->wall_normal, d), w = fabs(c) / ell;
  double sg = c < 0.0 ? -1.0 : 1.0;
  for (int i = 0; i < 3; ++i) dw_dd[i] = sg * S->wall_normal[i] / ell;
  *dw_dell = -w / ell;
  return w;
}

/* Radiance carried by one ray (the integrand of Eq. (2) for that sample) and its
   derivatives w.r.t. (u, v), the unit direction at the wall and the path length. */
static double ray_radiance(const or_scene* S, const double* uv, const double* d, double ell, int* tex, int lock,
                           double* dI, double* dId, double* dIp, int* off) {
  double L = wall_luminance(S, uv, tex, lock, dI, off);
  dId[0] = dId[1] = dId[2] = 0.0;
  *dIp = 0.0;
  if (!S->radiometry) return L;
  double dwd[3], dwp;
  double w = radiometric(S, d, ell, dwd, &dwp);
  dI[0] *= w;
  dI[1] *= w;
  for (int k = 0; k < 3; ++k) dId[k] = L * dwd[k];
  *dIp = L * dwp;
  return L * w;
}

int or_render_pixels(const or_scene* S, int32_t n_pixels, const double* uv, const double* vdir, const double* path,
                     uint8_t* status, double* image, double* dI_duv, double* dI_ddir, double* dI_dpath) {
  if (!S || !uv || !image || n_pixels < 0 || S->spp < 1 || !S->pattern || S->pat_w < 1 || S->pat_h < 1) return -1;
  if (S->radiometry && (!vdir || !path)) return -1;
  const int spp = S->spp;
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n_pixels; ++i) {
    double sum = 0.0;
    for (int s = 0; s < spp; ++s) {
      int64_t r = (int64_t)s * n_pixels + i;
      double dI[2] = {0.0, 0.0}, dId[3] = {0.0, 0.0, 0.0}, dIp = 0.0, I = 0.0;
      uint8_t st = status ? status[r] : 0;
      if (!(st & (OR_RAY_NO_WALL_HIT | OR_RAY_NONFINITE))) {
        int tex[2], off = 0;
        I = ray_radiance(S, &uv[2 * r], vdir ? &vdir[3 * r] : NULL, path ? path[r] : 0.0, tex, 0, dI, dId, &dIp,
                         &off);
        if (off && status) status[r] |= OR_RAY_OFF_PATTERN;
      }
      sum += I;
      if (dI_duv) { dI_duv[2 * r] = dI[0] / spp; dI_duv[2 * r + 1] = dI[1] / spp; }
      if (dI_ddir)
        for (int k = 0; k < 3; ++k) dI_ddir[3 * r + k] = dId[k] / spp;
      if (dI_dpath) dI_dpath[r] = dIp / spp;
    }
    image[i] = sum / spp;
  }
  return 0;
}

int or_loss_pixels(const double* image, const double* target, int32_t n_pixels, int32_t spp, const double* dI_duv,
                   const double* dI_ddir, const double* dI_dpath, double* loss, double* dL_duv, double* dL_ddir,
                   double* dL_dpath) {
  if (!image || !target || n_pixels < 0 || spp < 1) return -1;
  double L = 0.0;
  for (int32_t i = 0; i < n_pixels; ++i) {
    double res = image[i] - target[i];
    L += res * res;
    for (int s = 0; s < spp; ++s) {
      int64_t r = (int64_t)s * n_pixels + i;
      if (dL_duv && dI_duv) {
        dL_duv[2 * r] = 2.0 * res * dI_duv[2 * r];
        dL_duv[2 * r + 1] = 2.0 * res * dI_duv[2 * r + 1];
      }
      if (dL_ddir && dI_ddir)
        for (int k = 0; k < 3; ++k) dL_ddir[3 * r + k] = 2.0 * res * dI_ddir[3 * r + k];
      if (dL_dpath && dI_dpath) dL_dpath[r] = 2.0 * res * dI_dpath[r];
    }
  }
  if (loss) *loss = L;
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Sec. 2.D: exact gradient of the discrete forward map (reverse mode)                   */
/* ------------------------------------------------------------------------------------ */
static void voxel_index(const or_field* F, const cell_t* c, int a, int b, int k, int64_t* idx) {
  *idx = ((int64_t)(c->i0[2] + k) * F->n[1] + (c->i0[1] + b)) * F->n[0] + (c->i0[0] + a);
}

/* grad_c += scale * (dD/d delta_c) . q for the 8 corners of a sample, where
   dD/d delta_c = w_c grad(delta) + (1 + delta) grad(w_c). */
static void scatter_force(const or_field* F, const sample_t* s, const double* q, double scale, double* g) {
  double eta = 1.0 + s->delta;
  double gq = dot3(s->grad, q);
  for (int k = 0; k < 2; ++k)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        double wc = s->w[0][a] * s->w[1][b] * s->w[2][k];
        double gw[3] = {s->dw[0][a] * s->w[1][b] * s->w[2][k], s->w[0][a] * s->dw[1][b] * s->w[2][k],
                        s->w[0][a] * s->w[1][b] * s->dw[2][k]};
        int64_t idx;
        voxel_index(F, &s->cell, a, b, k, &idx);
        g[idx] += scale * (wc * gq + eta * dot3(gw, q));
      }
}

/* grad_c += scale * w_c (value derivative only). */
static void scatter_value(const or_field* F, const sample_t* s, double scale, double* g) {
  for (int k = 0; k < 2; ++k)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        int64_t idx;
        voxel_index(F, &s->cell, a, b, k, &idx);
        g[idx] += scale * s->w[0][a] * s->w[1][b] * s->w[2][k];
      }
}

/* dL/dx_n += lam_p (chat_{n-1} - chat_n) for a state 0 < n < N of the path polyline */
static void path_adjoint(const tape_t* tp, int n, double lam_p, double* rx) {
  if (lam_p == 0.0 || n == 0) return;
  double a[3], b[3];
  unit_from_to(&tp->x[3 * (n - 1)], &tp->x[3 * n], a);
  unit_from_to(&tp->x[3 * n], &tp->x[3 * (n + 1)], b);
  for (int i = 0; i < 3; ++i) rx[i] += lam_p * (a[i] - b[i]);
}

/* Reverse one ray given lambda = dL/d(u, v) (and dL/d direction, dL/d path length). */
static void adjoint_ray(const or_field* F, const or_scene* S, int32_t pix, int32_t sample, const double* lam_uv,
                        const double* lam_dir, double lam_p, tape_t* tp, double* g) {
  ray_result_t res;
  trace_ray(F, S, pix, sample, tp, 0, &res);
  if (!tp->entered) return;                                   /* straight camera ray */
  if (res.status & (OR_RAY_NO_WALL_HIT | OR_RAY_NONFINITE)) return; /* rendered as 0 */
  if (lam_uv[0] == 0.0 && lam_uv[1] == 0.0 && lam_p == 0.0 &&
      (!lam_dir || (lam_dir[0] == 0.0 && lam_dir[1] == 0.0 && lam_dir[2] == 0.0)))
    return;
  int N = tp->n_steps;
  double h = S->step;
  const double* xN = &tp->x[3 * N];
  const double* vN = &tp->v[3 * N];
  /* wall step: X = x + s v; dX/dx = I - v n^T/(v.n), dX/dv = s dX/dx */
  double X[3], s;
  wall_hit(S, xN, vN, X, &s);
  /* path = |x_0 - c| + sum_k |x_{k+1} - x_k| + s |v_N| with s |v_N| = (X - x_N).vhat_N:
     its variation is vhat_N.(dX - dx_N) (vhat_N . d vhat_N = 0), so it adds lam_p vhat_N
     to dL/dX and -lam_p vhat_N to dL/dx_N; every state k between adds
     lam_p (chat_{k-1} - chat_k) (chat_k the unit chord from x_k to x_{k+1}); x_0 is fixed
     by the camera */
  double vhat[3];
  {
    double len = sqrt(dot3(vN, vN));
    for (int i = 0; i < 3; ++i) vhat[i] = vN[i] / len;
  }
  double lX[3];
  for (int i = 0; i < 3; ++i) lX[i] = lam_uv[0] * S->wall_u[i] + lam_uv[1] * S->wall_v[i] + lam_p * vhat[i];
  double vn = dot3(vN, S->wall_normal), vl = dot3(vN, lX);
  double r[3], tau[3];
  for (int i = 0; i < 3; ++i) {
    r[i] = lX[i] - S->wall_normal[i] * vl / vn;
    tau[i] = s * r[i];
  }
  if (lam_p != 0.0) {
    double c_prev[3];
    unit_from_to(&tp->x[3 * (N - 1)], xN, c_prev);
    for (int i = 0; i < 3; ++i) r[i] += lam_p * (c_prev[i] - vhat[i]);
  }
  if (lam_dir) {
    /* the unit direction at the wall, d = v / |v|: dL/dv += (I - d d^T) dL/dd / |v| */
    double len = sqrt(dot3(vN, vN)), d[3];
    for (int i = 0; i < 3; ++i) d[i] = vN[i] / len;
    double dl = dot3(d, lam_dir);
    for (int i = 0; i < 3; ++i) tau[i] += (lam_dir[i] - d[i] * dl) / len;
  }
  const int quasi = S->tracer == OR_TRACER_QUASILINEAR;
  const double* x0 = &tp->x[0];
  const double* v0 = &tp->v[0];
  double lv0[3] = {0.0, 0.0, 0.0}; /* quasi-linear: dL/dv0 through the stage points on L */
  /* Sharma steps in reverse */
  for (int n = N - 1; n >= 0; --n) {
    stages_t st;
    double xn[3], vn2[3];
    ray_step(F, S, x0, v0, n, &tp->x[3 * n], &tp->v[3 * n], &tp->cells[1 + 3 * n], 1, xn, vn2, &st);
    double abar[3], bbar[3], cbar[3], rbar[3], tbar[3];
    for (int i = 0; i < 3; ++i) {
      abar[i] = h / 6.0 * r[i] + tau[i] / 6.0;
      bbar[i] = h / 3.0 * r[i] + 2.0 / 3.0 * tau[i];
      cbar[i] = tau[i] / 6.0;
      rbar[i] = r[i];
      tbar[i] = h * r[i] + tau[i];
    }
    double J[3][3], p[3];
    if (quasi) {
      /* stage points P_k = x0 + t_k v0 do not depend on the state: each stage adds its
         corner derivatives and t_k h J(P_k) bar_k to dL/dv0 */
      const double ts[3] = {n * h, n * h + 0.5 * h, n * h + h};
      const double* bars[3] = {abar, bbar, cbar};
      for (int k = 2; k >= 0; --k) {
        force_jacobian(&st.s[k], J);
        matvec3(J, bars[k], p);
        scatter_force(F, &st.s[k], bars[k], h, g);
        axpy3(lv0, ts[k] * h, p);
      }
      path_adjoint(tp, n, lam_p, rbar);
      memcpy(r, rbar, sizeof r);
      memcpy(tau, tbar, sizeof tau);
      continue;
    }
    /* stage C = h D(P3), P3 = x + h v + h/2 B */
    force_jacobian(&st.s[2], J);
    matvec3(J, cbar, p);
    for (int i = 0; i < 3; ++i) p[i] *= h;
    scatter_force(F, &st.s[2], cbar, h, g);
    axpy3(rbar, 1.0, p); axpy3(tbar, h, p); axpy3(bbar, 0.5 * h, p);
    /* stage B = h D(P2), P2 = x + h/2 v + h/8 A */
    force_jacobian(&st.s[1], J);
    matvec3(J, bbar, p);
    for (int i = 0; i < 3; ++i) p[i] *= h;
    scatter_force(F, &st.s[1], bbar, h, g);
    axpy3(rbar, 1.0, p); axpy3(tbar, 0.5 * h, p); axpy3(abar, 0.125 * h, p);
    /* stage A = h D(P1), P1 = x */
    force_jacobian(&st.s[0], J);
    matvec3(J, abar, p);
    for (int i = 0; i < 3; ++i) p[i] *= h;
    scatter_force(F, &st.s[0], abar, h, g);
    axpy3(rbar, 1.0, p);
    path_adjoint(tp, n, lam_p, rbar);
    memcpy(r, rbar, sizeof r);
    memcpy(tau, tbar, sizeof tau);
  }
  /* initial condition v_0 = (1 + delta(x_0)) d (quasi-linear: also the direction of L) */
  for (int i = 0; i < 3; ++i) tau[i] += lv0[i];
  sample_t s0;
  sample_field(F, tp->x0, &tp->cells[0], &s0);
  scatter_value(F, &s0, dot3(tau, tp->dir), g);
}

int or_adjoint(const or_field* F, const or_scene* S, const int32_t* pixel_ids, int32_t n_rays,
               const double* dL_duv, const double* dL_ddir, const double* dL_dpath, double* grad) {
  if (check_args(F, S, pixel_ids, n_rays) || F->mode != OR_FIELD_GRID || !dL_duv || !grad) return -1;
  int64_t nvox = (int64_t)F->n[0] * F->n[1] * F->n[2];
  int nth = omp_get_max_threads();
  double** part = (double**)calloc((size_t)nth, sizeof(double*));
  if (!part) return -3;
  int fail = 0;
#pragma omp parallel num_threads(nth)
  {
    int t = omp_get_thread_num();
    part[t] = (double*)calloc((size_t)nvox, sizeof(double));
    tape_t tp;
    int ok = part[t] && tape_init(&tp, S->max_steps);
    if (!ok) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp barrier
    if (!fail) {
#pragma omp for schedule(static, 16)
      for (int32_t r = 0; r < n_rays; ++r) {
        int32_t pix, sample;
        ray_pixel(S, pixel_ids, n_rays, r, &pix, &sample);
        adjoint_ray(F, S, pix, sample, &dL_duv[2 * r], dL_ddir ? &dL_ddir[3 * r] : NULL, dL_dpath ? dL_dpath[r] : 0.0,
                    &tp, part[t]);
      }
    }
    if (ok) tape_free(&tp);
  }
  if (!fail) {
    /* fixed summation order over threads -> deterministic for a given thread count */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nvox; ++i) {
      double acc = 0.0;
      for (int t = 0; t < nth; ++t) acc += part[t][i];
      grad[i] += acc;
    }
  }
  for (int t = 0; t < nth; ++t) free(part[t]);
  free(part);
  return fail ? -3 : 0;
}

/* ------------------------------------------------------------------------------------ */
/* Tangent-linear model (forward-mode derivative of the same discrete map)               */
/* ------------------------------------------------------------------------------------ */
/* dD = J dP + (dDelta grad(delta) + (1 + delta) grad(dDelta)) for a field perturbation vf */
static void force_tangent(const or_field* F, const sample_t* s, const double* dP, const double* vf, double* dD) {
  double J[3][3];
  force_jacobian(s, J);
  matvec3(J, dP, dD);
  double dd = 0.0, gd[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 2; ++k)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        int64_t idx;
        voxel_index(F, &s->cell, a, b, k, &idx);
        double val = vf[idx];
        dd += s->w[0][a] * s->w[1][b] * s->w[2][k] * val;
        gd[0] += s->dw[0][a] * s->w[1][b] * s->w[2][k] * val;
        gd[1] += s->w[0][a] * s->dw[1][b] * s->w[2][k] * val;
        gd[2] += s->w[0][a] * s->w[1][b] * s->dw[2][k] * val;
      }
  double eta = 1.0 + s->delta;
  for (int i = 0; i < 3; ++i) dD[i] += dd * s->grad[i] + eta * gd[i];
}

static void tangent_ray(const or_field* F, const or_scene* S, int32_t pix, int32_t sample, const double* vf,
                        tape_t* tp, double* out, double* out_dir, double* out_path) {
  ray_result_t res;
  trace_ray(F, S, pix, sample, tp, 0, &res);
  out[0] = out[1] = 0.0;
  if (out_dir) out_dir[0] = out_dir[1] = out_dir[2] = 0.0;
  if (out_path) *out_path = 0.0;
  double dpath = 0.0; /* sum_k chat_k . (dx_{k+1} - dx_k), dx_0 = 0 */
  if (!tp->entered || (res.status & (OR_RAY_NO_WALL_HIT | OR_RAY_NONFINITE))) return;
  double h = S->step;
  sample_t s0;
  sample_field(F, tp->x0, &tp->cells[0], &s0);
  double dd0 = 0.0;
  for (int k = 0; k < 2; ++k)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        int64_t idx;
        voxel_index(F, &s0.cell, a, b, k, &idx);
        dd0 += s0.w[0][a] * s0.w[1][b] * s0.w[2][k] * vf[idx];
      }
  double dx[3] = {0.0, 0.0, 0.0}, dv[3], dv0[3];
  for (int i = 0; i < 3; ++i) dv[i] = dv0[i] = dd0 * tp->dir[i];
  const int quasi = S->tracer == OR_TRACER_QUASILINEAR;
  for (int n = 0; n < tp->n_steps; ++n) {
    stages_t st;
    double xn[3], vn[3], dA[3], dB[3], dC[3], dP[3], dD[3];
    ray_step(F, S, &tp->x[0], &tp->v[0], n, &tp->x[3 * n], &tp->v[3 * n], &tp->cells[1 + 3 * n], 1, xn, vn,
             &st);
    if (quasi) {
      /* stage points x0 + t_k v0 move with v0 only */
      double* dK[3] = {dA, dB, dC};
      const double ts[3] = {n * h, n * h + 0.5 * h, n * h + h};
      for (int k = 0; k < 3; ++k) {
        for (int i = 0; i < 3; ++i) dP[i] = ts[k] * dv0[i];
        force_tangent(F, &st.s[k], dP, vf, dD);
        for (int i = 0; i < 3; ++i) dK[k][i] = h * dD[i];
      }
      double c[3], dx_old[3];
      memcpy(dx_old, dx, sizeof dx);
      for (int i = 0; i < 3; ++i) {
        dx[i] = dx[i] + h * (dv[i] + (dA[i] + 2.0 * dB[i]) / 6.0);
        dv[i] = dv[i] + (dA[i] + 4.0 * dB[i] + dC[i]) / 6.0;
      }
      unit_from_to(&tp->x[3 * n], &tp->x[3 * (n + 1)], c);
      for (int i = 0; i < 3; ++i) dpath += c[i] * (dx[i] - dx_old[i]);
      continue;
    }
    force_tangent(F, &st.s[0], dx, vf, dD);
    for (int i = 0; i < 3; ++i) dA[i] = h * dD[i];
    for (int i = 0; i < 3; ++i) dP[i] = dx[i] + 0.5 * h * dv[i] + 0.125 * h * dA[i];
    force_tangent(F, &st.s[1], dP, vf, dD);
    for (int i = 0; i < 3; ++i) dB[i] = h * dD[i];
    for (int i = 0; i < 3; ++i) dP[i] = dx[i] + h * dv[i] + 0.5 * h * dB[i];
    force_tangent(F, &st.s[2], dP, vf, dD);
    for (int i = 0; i < 3; ++i) dC[i] = h * dD[i];
    double c[3], dx_old[3];
    memcpy(dx_old, dx, sizeof dx);
    for (int i = 0; i < 3; ++i) {
      dx[i] = dx[i] + h * (dv[i] + (dA[i] + 2.0 * dB[i]) / 6.0);
      dv[i] = dv[i] + (dA[i] + 4.0 * dB[i] + dC[i]) / 6.0;
    }
    unit_from_to(&tp->x[3 * n], &tp->x[3 * (n + 1)], c);
    for (int i = 0; i < 3; ++i) dpath += c[i] * (dx[i] - dx_old[i]);
  }
  const double* x = &tp->x[3 * tp->n_steps];
  const double* v = &tp->v[3 * tp->n_steps];
  double X[3], s;
  wall_hit(S, x, v, X, &s);
  double vn = dot3(v, S->wall_normal);
  double ds = -dot3(dx, S->wall_normal) / vn - s * dot3(dv, S->wall_normal) / vn;
  double dX[3];
  for (int i = 0; i < 3; ++i) dX[i] = dx[i] + ds * v[i] + s * dv[i];
  out[0] = dot3(dX, S->wall_u);
  out[1] = dot3(dX, S->wall_v);
  if (out_path) {
    double len = sqrt(dot3(v, v)), vhat[3];
    for (int i = 0; i < 3; ++i) vhat[i] = v[i] / len;
    *out_path = dpath + dot3(vhat, dX) - dot3(vhat, dx);
  }
  if (out_dir) {
    /* d = v / |v|: dd = (I - d d^T) dv / |v| */
    double len = sqrt(dot3(v, v)), d[3];
    for (int i = 0; i < 3; ++i) d[i] = v[i] / len;
    double dd = dot3(d, dv);
    for (int i = 0; i < 3; ++i) out_dir[i] = (dv[i] - d[i] * dd) / len;
  }
}

int or_tangent(const or_field* F, const or_scene* S, const int32_t* pixel_ids, int32_t n_rays,
               const double* vfield, double* duv_dot, double* ddir_dot, double* dpath_dot) {
  if (check_args(F, S, pixel_ids, n_rays) || F->mode != OR_FIELD_GRID || !vfield || !duv_dot) return -1;
  int fail = 0;
#pragma omp parallel
  {
    tape_t tp;
    int ok = tape_init(&tp, S->max_steps);
    if (!ok) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int32_t r = 0; r < n_rays; ++r) {
      if (!ok) continue;
      int32_t pix, sample;
      ray_pixel(S, pixel_ids, n_rays, r, &pix, &sample);
      tangent_ray(F, S, pix, sample, vfield, &tp, &duv_dot[2 * r], ddir_dot ? &ddir_dot[3 * r] : NULL,
                  dpath_dot ? &dpath_dot[r] : NULL);
    }
    if (ok) tape_free(&tp);
  }
  return fail ? -3 : 0;
}

/* ------------------------------------------------------------------------------------ */
/* Central finite differences of L_BOS with respect to single voxels                     */
/* ------------------------------------------------------------------------------------ */
/* Radiance of one ray (its sample of Eq. (2)), optionally replaying a tape. */
static double ray_value(const or_field* F, const or_scene* S, int32_t pix, int32_t sample, tape_t* tp, int locked,
                        int* tex) {
  ray_result_t res;
  trace_ray(F, S, pix, sample, tp, locked, &res);
  if (res.status & (OR_RAY_NO_WALL_HIT | OR_RAY_NONFINITE)) return 0.0;
  double dI[2], dId[3], dIp, d[3];
  int off;
  double len = sqrt(dot3(res.v, res.v));
  for (int i = 0; i < 3; ++i) d[i] = res.v[i] / len;
  return ray_radiance(S, res.uv, d, res.path, tex, locked, dI, dId, &dIp, &off);
}

static int ray_touches(const or_field* F, const tape_t* tp, int64_t vox) {
  if (!tp->entered) return 0;
  int nx = F->n[0], ny = F->n[1];
  int vi = (int)(vox % nx), vj = (int)((vox / nx) % ny), vk = (int)(vox / ((int64_t)nx * ny));
  int ns = 1 + 3 * tp->n_steps;
  for (int k = 0; k < ns; ++k) {
    const cell_t* c = &tp->cells[k];
    if (vi - c->i0[0] >= 0 && vi - c->i0[0] <= 1 && vj - c->i0[1] >= 0 && vj - c->i0[1] <= 1 &&
        vk - c->i0[2] >= 0 && vk - c->i0[2] <= 1)
      return 1;
  }
  return 0;
}

int or_fd_voxels(const or_field* F, const or_scene* S, const int32_t* pixel_ids, int32_t n_rays,
                 const double* target, const int64_t* voxels, int32_t n_vox, double h, int32_t locked,
                 double* fd) {
  if (check_args(F, S, pixel_ids, n_rays) || F->mode != OR_FIELD_GRID || !target || !voxels || !fd ||
      n_vox < 0 || n_vox > 64 || !(h > 0.0) || !S->pattern)
    return -1;
  const int32_t spp = S->spp, P = n_rays / spp;
  /* pass 1: which pixels (through any of their rays) can see which voxel */
  uint64_t* mask = (uint64_t*)calloc((size_t)(P > 0 ? P : 1), sizeof(uint64_t));
  if (!mask) return -3;
  int fail = 0;
#pragma omp parallel
  {
    tape_t tp;
    int ok = tape_init(&tp, S->max_steps);
    if (!ok) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 64)
    for (int32_t i = 0; i < P; ++i) {
      if (!ok) continue;
      int32_t pix = pixel_ids ? pixel_ids[i] : i;
      uint64_t m = 0;
      for (int32_t smp = 0; smp < spp; ++smp) {
        ray_result_t res;
        trace_ray(F, S, pix, smp, &tp, 0, &res);
        for (int v = 0; v < n_vox; ++v)
          if (ray_touches(F, &tp, voxels[v])) m |= (uint64_t)1 << v;
      }
      mask[i] = m;
    }
    if (ok) tape_free(&tp);
  }
  if (fail) { free(mask); return -3; }
  /* pass 2: perturbed pixel values (all samples) of the touching pixels only */
  for (int v = 0; v < n_vox; ++v) {
    double acc = 0.0;
#pragma omp parallel reduction(+ : acc)
    {
      tape_t tp;
      int ok = tape_init(&tp, S->max_steps);
      or_field Fp = *F, Fm = *F;
      Fp.pert_index = voxels[v]; Fp.pert_value = h;
      Fm.pert_index = voxels[v]; Fm.pert_value = -h;
#pragma omp for schedule(dynamic, 8)
      for (int32_t i = 0; i < P; ++i) {
        if (!ok || !(mask[i] >> v & 1)) continue;
        int32_t pix = pixel_ids ? pixel_ids[i] : i;
        double Ip = 0.0, Im = 0.0;
        for (int32_t smp = 0; smp < spp; ++smp) {
          int tex[2];
          if (locked) {
            (void)ray_value(F, S, pix, smp, &tp, 0, tex); /* record branches */
            Ip += ray_value(&Fp, S, pix, smp, &tp, 1, tex);
            Im += ray_value(&Fm, S, pix, smp, &tp, 1, tex);
          } else {
            Ip += ray_value(&Fp, S, pix, smp, NULL, 0, tex);
            Im += ray_value(&Fm, S, pix, smp, NULL, 0, tex);
          }
        }
        double rp = Ip / spp - target[i], rm = Im / spp - target[i];
        acc += rp * rp - rm * rm;
      }
      if (ok) tape_free(&tp);
    }
    fd[v] = acc / (2.0 * h);
  }
  free(mask);
  return 0;
}
