// particles.hpp -- push and deposit kernels, FP64 form and single-precision form.
//
// One particle per lane; structure-of-arrays loads and stores are contiguous
// across a wavefront.  The push follows Sec. 3.1 steps 1-11 of the paper; the
// deposit Sec. 3.2.  The single-precision form stores cell indices as int32
// and offsets, momenta, fields and currents as float, evaluates the metric in
// float from offsets relative to the particle's cell (angles from the nearer
// axis), and takes the metric and its derivatives at x^n in FP64 inside the
// horizon region (cells i1 < i_fp64).
#pragma once

#include <type_traits>

#include <climits>

#include "geometry.hpp"

namespace grpic {

constexpr uint8_t kLeaving = 0x80;
constexpr uint8_t kInvalid = 0x40;  // dropped by a bounds guard; never used again
constexpr uint8_t kSpecies = 0x03;
constexpr uint8_t kMassless = 0x04;  // with species 3: a massless neutral particle

__host__ __device__ inline bool is_live(uint8_t t) { return t != 0 && !(t & kInvalid); }

// m^2 in gamma = sqrt(m^2 + h^ij u_i u_j) (Sec. 2.3): 0 for a massless neutral
// particle (species 3 with the massless bit), 1 otherwise
__host__ __device__ inline double mass2_of(uint8_t t) {
  return (t & (kSpecies | kMassless)) == (kSpecies | kMassless) ? 0.0 : 1.0;
}

// a position inside the grid (what the push may start from)
template <class T>
__device__ inline bool in_grid(const Grid& g, int i1, T dx1, int i2, T dx2) {
  return i1 >= 0 && i1 < g.n_r && i2 >= 0 && i2 < g.n_th && dx1 >= (T)0 && dx1 <= (T)1 &&
         dx2 >= (T)0 && dx2 <= (T)1;
}

// a position the deposit may write around: one cell beyond the radial edges
template <class T>
__device__ inline bool in_deposit_range(const Grid& g, int i1, T dx1, int i2, T dx2) {
  return i1 >= -1 && i1 <= g.n_r && i2 >= 0 && i2 < g.n_th && dx1 >= (T)0 && dx1 <= (T)1 &&
         dx2 >= (T)0 && dx2 <= (T)1;
}

template <class T>
struct ParticleArraysT {
  int32_t* __restrict__ i1;
  int32_t* __restrict__ i2;
  T* __restrict__ dx1;
  T* __restrict__ dx2;
  T* __restrict__ u1;
  T* __restrict__ u2;
  T* __restrict__ u3;
  T* __restrict__ w;
  T* __restrict__ phi;
  int32_t* __restrict__ i1p;
  int32_t* __restrict__ i2p;
  T* __restrict__ dx1p;
  T* __restrict__ dx2p;
  uint8_t* __restrict__ tag;
  int64_t n;
};
using ParticleArrays = ParticleArraysT<double>;

template <class T>
struct GatherPlanesT {
  const T* __restrict__ D[3];
  const T* __restrict__ B[3];
};

__device__ inline double species_sign(uint8_t t) {
  const int s = t & kSpecies;
  return s == 1 ? 1.0 : (s == 2 ? -1.0 : 0.0);
}

// First-order interpolation in code coordinates of a plane staggered by half a
// cell in x1 (H1) and/or x2 (H2).
template <int H1, int H2, class T>
__device__ inline T interp(const Grid& g, const T* __restrict__ F, int i1, T dx1, int i2, T dx2) {
  int k1 = i1, k2 = i2;
  T w1 = dx1, w2 = dx2;
  const T half = (T)0.5;
  if (H1) {
    const bool up = dx1 >= half;
    k1 = up ? i1 : i1 - 1;
    w1 = up ? dx1 - half : dx1 + half;
  }
  if (H2) {
    const bool up = dx2 >= half;
    k2 = up ? i2 : i2 - 1;
    w2 = up ? dx2 - half : dx2 + half;
  }
  const T* p = F + ix(g, k1, k2);
  const T f00 = p[0], f01 = p[1], f10 = p[g.ld], f11 = p[g.ld + 1];
  const T a0 = f00 + w2 * (f01 - f00);
  const T a1 = f10 + w2 * (f11 - f10);
  return a0 + w1 * (a1 - a0);
}

// Relativistic Boris step for duration tau in an orthonormal frame: u_minus
// = u + k E, the rotation (u_minus + u_minus x t) x s, the second electric
// half kick.  Returns the change of u (both kicks plus the rotation term).
template <class R>
__device__ inline void boris_delta(R ux, R uy, R uz, const R E[3], const R B[3], R k /* = qm tau / 2 */,
                                   R& dx, R& dy, R& dz) {
  // (single precision: reciprocal and reciprocal square root from the
  // hardware seeds with a Newton step, about an ulp, in place of the
  // correctly rounded division and square root)
  const R mx = ux + k * E[0], my = uy + k * E[1], mz = uz + k * E[2];
  const R ig = k * rsqrt((R)1 + mx * mx + my * my + mz * mz);
  const R tx = B[0] * ig, ty = B[1] * ig, tz = B[2] * ig;
  const R f = (R)2 * rcp((R)1 + tx * tx + ty * ty + tz * tz);
  const R sx = f * tx, sy = f * ty, sz = f * tz;
  const R px = mx + (my * tz - mz * ty);
  const R py = my + (mz * tx - mx * tz);
  const R pz = mz + (mx * ty - my * tx);
  const R k2 = k + k;
  dx = (py * sz - pz * sy) + k2 * E[0];
  dy = (pz * sx - px * sz) + k2 * E[1];
  dz = (px * sy - py * sx) + k2 * E[2];
}

// The same Boris step applied to u in place (reciprocal and reciprocal square
// root as in boris_delta; in double precision two Newton steps, about an ulp).
template <class R>
__device__ inline void boris(R& ux, R& uy, R& uz, const R E[3], const R B[3], R k /* = qm tau / 2 */) {
  const R mx = ux + k * E[0], my = uy + k * E[1], mz = uz + k * E[2];
  const R ig = k * rsqrt((R)1 + mx * mx + my * my + mz * mz);
  const R tx = B[0] * ig, ty = B[1] * ig, tz = B[2] * ig;
  const R f = (R)2 * rcp((R)1 + tx * tx + ty * ty + tz * tz);
  const R sx = f * tx, sy = f * ty, sz = f * tz;
  const R px = mx + (my * tz - mz * ty);
  const R py = my + (mz * tx - mx * tz);
  const R pz = mz + (mx * ty - my * tx);
  ux = mx + (py * sz - pz * sy) + k * E[0];
  uy = my + (pz * sx - px * sz) + k * E[1];
  uz = mz + (px * sy - py * sx) + k * E[2];
}

// EM half step: covariant -> tetrad (App. A), Boris, tetrad -> covariant.
// Single precision takes only the change of the tetrad components back and
// adds it to the covariant u, so u carries one rounding per half step instead
// of those of a full round trip through the tetrad (which would dominate the
// error of the single-precision form over many steps).  Double precision
// (and the adjoint's tangent numbers) take the whole vector back: the round
// trip costs nothing visible there, and it keeps fewer values live.
template <class R>
__device__ inline void em_half(const FrameT<R>& f, const R E[3], const R B[3], R k, R& u1, R& u2,
                               R& u3) {
  if constexpr (sizeof(R) == 4) {
    const R x = f.s11 * (u1 - f.k13 * u3);
    const R y = u2 * rcp(f.s22);
    const R z = u3 * rcp(f.s33);
    R dx, dy, dz;
    boris_delta(x, y, z, E, B, k, dx, dy, dz);
    u1 = u1 + (dx * rcp(f.s11) + f.k13 * f.s33 * dz);
    u2 = u2 + f.s22 * dy;
    u3 = u3 + f.s33 * dz;
  } else {
    R x = f.s11 * (u1 - f.k13 * u3);
    R y = u2 / f.s22;
    R z = u3 / f.s33;
    boris(x, y, z, E, B, k);
    u1 = x / f.s11 + f.k13 * f.s33 * z;
    u2 = f.s22 * y;
    u3 = f.s33 * z;
  }
}

// Implicit-midpoint geodesic momentum update at fixed x^n (eq.
// discretized-geodesic-u); u_3 is untouched.
template <class R>
__device__ inline void geodesic_u(const Grid& g, const FrameT<R>& f, const GradT<R>& d, R& u1, R& u2,
                                  R u3, R mass2) {
  const CoeffsT<R>& m = f.c;
  const R s1 = u1, s2 = u2;
  const R u33 = u3 * u3;
  const R dt = (R)g.dt;
  R t1 = s1, t2 = s2;
  for (int it = 0; it < g.n_iter; ++it) {
    const R b1 = (R)0.5 * (s1 + t1), b2 = (R)0.5 * (s2 + t2);
    const R Q = mass2 + m.hu11 * b1 * b1 + m.hu22 * b2 * b2 + m.hu33 * u33 + (R)2 * m.hu13 * b1 * u3;
    const R ig = rsqrt(Q);
    const R gb = Q * ig;
    const R h = (R)0.5 * m.alpha * ig;
    R fr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const R q = d.hu11[i] * b1 * b1 + d.hu22[i] * b2 * b2 + d.hu33[i] * u33 +
                  (R)2 * d.hu13[i] * b1 * u3;
      fr[i] = -gb * d.alpha[i] + b1 * d.beta1[i] - h * q;
    }
    const R n1 = s1 + dt * fr[0], n2 = s2 + dt * fr[1];
    // exact repeat: the fixed point of the map; or the optional convergence
    // test, evaluated in FP64
    bool fixed = n1 == t1 && n2 == t2;
    if (g.iter_tol > 0.0)
      fixed = fixed || fabs((double)n1 - (double)t1) + fabs((double)n2 - (double)t2) <=
                           g.iter_tol * (fabs((double)n1) + fabs((double)n2));
    t1 = n1;
    t2 = n2;
    if (fixed) break;
  }
  u1 = t1;
  u2 = t2;
}

template <class R>
__device__ inline void renormalize(int& i, R& dx) {
  const R f = floor(dx);
  i += (int)f;
  dx -= f;
  if (dx >= (R)1) {
    dx -= (R)1;
    i += 1;
  }
}

// exp(t) for |t| <= 0.11: Taylor series to t^11 (remainder below 1e-20 relative)
__device__ inline double exp_small(double t) {
  double p = fma(t, 1.0 / 39916800.0, 1.0 / 3628800.0);
  p = fma(t, p, 1.0 / 362880.0);
  p = fma(t, p, 1.0 / 40320.0);
  p = fma(t, p, 1.0 / 5040.0);
  p = fma(t, p, 1.0 / 720.0);
  p = fma(t, p, 1.0 / 120.0);
  p = fma(t, p, 1.0 / 24.0);
  p = fma(t, p, 1.0 / 6.0);
  p = fma(t, p, 0.5);
  p = fma(t, p, 1.0);
  return fma(t, p, 1.0);
}

// sin and cos for |x| <= 0.11: Taylor series to x^13 and x^14
__device__ inline void sincos_small(double x, double* s, double* c) {
  const double z = x * x;
  double ps = fma(z, 1.0 / 6227020800.0, -1.0 / 39916800.0);
  ps = fma(z, ps, 1.0 / 362880.0);
  ps = fma(z, ps, -1.0 / 5040.0);
  ps = fma(z, ps, 1.0 / 120.0);
  ps = fma(z, ps, -1.0 / 6.0);
  *s = fma(x * z, ps, x);
  double pc = fma(z, -1.0 / 87178291200.0, 1.0 / 479001600.0);
  pc = fma(z, pc, -1.0 / 3628800.0);
  pc = fma(z, pc, 1.0 / 40320.0);
  pc = fma(z, pc, -1.0 / 720.0);
  pc = fma(z, pc, 1.0 / 24.0);
  pc = fma(z, pc, -0.5);
  *c = fma(z, pc, 1.0);
}

// exp(t) for |t| <= 0.03: Taylor series to t^8 (remainder below 1e-19 relative)
__device__ inline double exp_short(double t) {
  double p = fma(t, 1.0 / 40320.0, 1.0 / 5040.0);
  p = fma(t, p, 1.0 / 720.0);
  p = fma(t, p, 1.0 / 120.0);
  p = fma(t, p, 1.0 / 24.0);
  p = fma(t, p, 1.0 / 6.0);
  p = fma(t, p, 0.5);
  p = fma(t, p, 1.0);
  return fma(t, p, 1.0);
}

// sin and cos for |x| <= 0.03: Taylor series to x^7 and x^6 (remainders
// below 2e-17 relative)
__device__ inline void sincos_short(double x, double* s, double* c) {
  const double z = x * x;
  double ps = fma(z, -1.0 / 5040.0, 1.0 / 120.0);
  ps = fma(z, ps, -1.0 / 6.0);
  *s = fma(x * z, ps, x);
  double pc = fma(z, -1.0 / 720.0, 1.0 / 24.0);
  pc = fma(z, pc, -0.5);
  *c = fma(z, pc, 1.0);
}

// pi - (pi rounded to double)
constexpr double kPiLo = 1.2246467991473531772e-16;

// r, sin, cos and the map factors at code position (x1, x2) near cell
// (i1, i2) (|x - i| <= 1.5) on the logarithmic-r, uniform-theta grid:
// r = r_i exp((x1 - i1) dxi); the polar angle is first rounded and clamped as
// theta = clamp(x2 dth), and the result is the sine and cosine of that double:
// by a series on theta itself next to theta = 0, on psi = pi - theta (exact
// subtraction plus the low part of pi) next to theta = pi, so that sin keeps
// its relative precision next to both axes (within the band, angle addition
// would cancel), and by angle addition from the tables elsewhere.
// SER = 2: offsets |x - i| dxi, dth <= 0.03 and an axis band of 4 cells (its
// angles <= 0.03): short series throughout.  SER = 1: offsets <= 0.11 and an
// axis band of 0.11 rad: long series.  SER = 0: library functions (also every
// general quasi-spherical map).
template <int SER>
__device__ inline RSC rsc_near(const Grid& g, const Tables& t, int i1, double x1, int i2, double x2) {
  if (SER == 0) return rsc_direct(g, x1, x2);
  RSC p;
  const double tr = (x1 - (double)i1) * g.dxi;
  p.r = t.r[0][i1 + g.ng] * (SER == 2 ? exp_short(tr) : exp_small(tr));
  p.rd = g.dxi * p.r;
  p.td = g.dth;
  p.itd2 = g.inv_dth2;
  p.dtd = 0.0;
  const double th = x2 * g.dth;
  const double band = SER == 2 ? g.axis_band : 0.11;
  if (th <= g.small_angle) {
    p.s = g.sin_lo;
    p.c = g.cos_lo;
  } else if (th >= g.th_hi) {
    p.s = g.sin_hi;
    p.c = g.cos_hi;
  } else if (th <= band) {
    if (SER == 2) sincos_short(th, &p.s, &p.c); else sincos_small(th, &p.s, &p.c);
  } else if (th >= (SER == 2 ? g.band_hi : kPi - 0.11)) {
    double cq;
    if (SER == 2) sincos_short((kPi - th) + kPiLo, &p.s, &cq);
    else sincos_small((kPi - th) + kPiLo, &p.s, &cq);
    p.c = -cq;
  } else {
    double sp, cp;
    if (SER == 2) sincos_short(th - (double)i2 * g.dth, &sp, &cp);
    else sincos_small(th - (double)i2 * g.dth, &sp, &cp);
    const double sj = t.s[0][i2 + g.ng], cj = t.c[0][i2 + g.ng];
    p.s = fma(sj, cp, cj * sp);
    p.c = fma(cj, cp, -(sj * sp));
  }
  return p;
}

// single-precision series for |x| <= 0.11 (truncation below 1e-9 relative)
__device__ inline float exp_small_f(float t) {
  float p = fmaf(t, 1.0f / 720.0f, 1.0f / 120.0f);
  p = fmaf(t, p, 1.0f / 24.0f);
  p = fmaf(t, p, 1.0f / 6.0f);
  p = fmaf(t, p, 0.5f);
  p = fmaf(t, p, 1.0f);
  return fmaf(t, p, 1.0f);
}

__device__ inline void sincos_small_f(float x, float* s, float* c) {
  const float z = x * x;
  float ps = fmaf(z, -1.0f / 5040.0f, 1.0f / 120.0f);
  ps = fmaf(z, ps, -1.0f / 6.0f);
  *s = fmaf(x * z, ps, x);
  float pc = fmaf(z, 1.0f / 40320.0f, -1.0f / 720.0f);
  pc = fmaf(z, pc, 1.0f / 24.0f);
  pc = fmaf(z, pc, -0.5f);
  *c = fmaf(z, pc, 1.0f);
}

// Single precision: r, sin, cos and the map factors at offsets (f1, f2) from
// the corner of cell (i1, i2), |f| <= 1.5.  The polar angle is measured from
// the nearer axis, theta(x2) or pi - theta(x2) = theta(n_th - x2) (the map is
// symmetric about the equator), so that sin keeps its relative precision next
// to either axis; clamped at small_angle.  SER > 0: the logarithmic-r,
// uniform-theta grid with series; SER = 0: the general map of App. A with the
// library functions.
template <int SER>
__device__ inline RSCT<float> rsc_near_f(const Grid& g, const Tables& t, int i1, float f1, int i2,
                                        float f2) {
  RSCT<float> p;
  const float dth = (float)g.dth, eps = (float)g.small_angle;
  const float e = SER > 0 ? t.rf[i1 + g.ng] * exp_small_f(f1 * (float)g.dxi)
                          : t.rf[i1 + g.ng] * expf(f1 * (float)g.dxi);
  p.r = SER > 0 ? e : (float)g.r0 + e;
  p.rd = (float)g.dxi * e;
  const bool upper = 2 * i2 >= g.n_th;
  const float eta = upper ? ((float)(g.n_th - i2) - f2) * dth : ((float)i2 + f2) * dth;
  float ang = eta;
  if (SER > 0) {
    p.td = dth;
    p.itd2 = (float)g.inv_dth2;
    p.dtd = 0.0f;
  } else {
    // past the axis (a midpoint of the coordinate iteration) the map is
    // continued by reflection, as in map_theta: theta odd, T even, dT odd
    const bool past = eta < 0.0f;
    const float ea = past ? -eta : eta;
    const float h0 = (float)g.h0, pi = (float)kPi, y = ea * (float)(1.0 / kPi);
    const float th = ea + 2.0f * h0 * ea * (pi - 2.0f * ea) * (pi - ea) * (float)(1.0 / (kPi * kPi));
    ang = past ? -th : th;
    p.td = dth * (1.0f + 2.0f * h0 + 12.0f * h0 * y * (y - 1.0f));
    p.itd2 = rcp(p.td * p.td);
    const float dd = dth * dth * 12.0f * h0 * (2.0f * y - 1.0f) * (float)(1.0 / kPi);
    p.dtd = (upper != past) ? -dd : dd;
  }
  float s, c;
  if (ang <= eps) {
    s = (float)g.sin_lo;
    c = (float)g.cos_lo;
  } else if (SER == 0) {
    sincosf(ang, &s, &c);
  } else if (ang <= 0.11f) {
    sincos_small_f(ang, &s, &c);
  } else {
    // angle addition about the table node theta_i2 (float tables)
    float sp, cp;
    sincos_small_f(f2 * dth, &sp, &cp);
    const float sj = t.sf[i2 + g.ng], cj = t.cf[i2 + g.ng];
    p.s = fmaf(sj, cp, cj * sp);
    p.c = fmaf(cj, cp, -(sj * sp));
    return p;
  }
  p.s = s;
  p.c = upper ? -c : c;
  return p;
}

// Sort key of a slot's state: its cell i1 * n_th + i2, or n_cells for a slot
// that the cell sort drops (empty, invalid, leaving, outside the grid).
__device__ inline int cell_key(const Grid& g, uint8_t t, int i1, int i2) {
  if (!is_live(t) || (t & kLeaving) || i1 < 0 || i1 >= g.n_r || i2 < 0 || i2 >= g.n_th) return g.n_r * g.n_th;
  return i1 * g.n_th + i2;
}

// What the deposit needs from one particle's move (Sec. 3.2).
template <class T>
struct Move {
  bool dep;            // deposits a current this step
  bool mid;            // vphi holds alpha u^3 / gamma at the deposit's path midpoint
  int ia, ja, ib, jb;  // previous and current cell
  T xa, ya, xb, yb;    // previous and current offsets
  T q;                 // species sign x charge_scale x weight
  T vphi;
  T u1, u2, u3;        // u^{n+1/2}, for vphi when !mid
  int cell;            // sort key of the state after the push (cell_key)
};

// FP64 particle update (Sec. 3.1 steps 1-11) of slot k; writes the new state
// and returns the move for the deposit.
template <int SER, bool kPrev = true>
__device__ inline Move<double> push_one(const Grid& g, const Tables& tab, const GatherPlanesT<double>& fp,
                                        const ParticleArrays& P, int64_t k) {
  Move<double> mv;
  mv.dep = false;
  mv.cell = g.n_r * g.n_th;
  if (k >= P.n) return mv;
  uint8_t t = P.tag[k];
  if (!is_live(t)) return mv;
  if (t & kLeaving) {
    P.tag[k] = 0;
    return mv;
  }
  int i1 = P.i1[k], i2 = P.i2[k];
  double dx1 = P.dx1[k], dx2 = P.dx2[k];
  if (!in_grid(g, i1, dx1, i2, dx2)) {  // corrupt input: drop, never index with it
    P.tag[k] = kInvalid;
    return mv;
  }
  double u1 = P.u1[k], u2 = P.u2[k], u3 = P.u3[k];
  if (kPrev) {  // the previous position, for a separate deposit
    P.i1p[k] = i1;
    P.i2p[k] = i2;
    P.dx1p[k] = dx1;
    P.dx2p[k] = dx2;
  }
  mv.ia = i1;
  mv.ja = i2;
  mv.xa = dx1;
  mv.ya = dx2;

  const double x1 = (double)i1 + dx1, x2 = (double)i2 + dx2;
  Frame f;
  Grad d;
  frame_from(g, rsc_near<SER>(g, tab, i1, x1, i2, x2), &f, &d);
  const double qm = species_sign(t);
  if (qm != 0.0) {
    // D^i, B^i at x^n -> tetrad components, scaled by the lapse
    const double D1 = interp<1, 0>(g, fp.D[0], i1, dx1, i2, dx2);
    const double D2 = interp<0, 1>(g, fp.D[1], i1, dx1, i2, dx2);
    const double D3 = interp<0, 0>(g, fp.D[2], i1, dx1, i2, dx2);
    const double B1 = interp<0, 1>(g, fp.B[0], i1, dx1, i2, dx2);
    const double B2 = interp<1, 0>(g, fp.B[1], i1, dx1, i2, dx2);
    const double B3 = interp<1, 1>(g, fp.B[2], i1, dx1, i2, dx2);
    const double al = f.c.alpha, ais11 = al * rcp(f.s11);
    const double E[3] = {ais11 * D1, al * f.s22 * D2, al * f.s33 * (f.k13 * D1 + D3)};
    const double B[3] = {ais11 * B1, al * f.s22 * B2, al * f.s33 * (f.k13 * B1 + B3)};
    const double kb = 0.25 * qm * g.dt;
    em_half(f, E, B, kb, u1, u2, u3);
    geodesic_u(g, f, d, u1, u2, u3, 1.0);
    em_half(f, E, B, kb, u1, u2, u3);
  } else {
    geodesic_u(g, f, d, u1, u2, u3, mass2_of(t));  // EM stage skipped for q = 0
  }

  // implicit coordinate update (eq. discretized-geodesic-x); an iterate that
  // repeats exactly is the fixed point of the map, so stopping there gives the
  // same result as running all n_iter iterations (and with iter_tol > 0 the
  // loop also ends once the FP64 change is below the relative tolerance)
  // The first iterate (d = 0) uses the coefficients at x^n already in hand.
  double d1 = 0.0, d2 = 0.0;
  Coeffs m = f.c;
  // m^2 from the tag, taken here rather than at the top: the empty asm keeps
  // the compiler from hoisting it, so that it is not live through the field
  // gather and EM stages, where the FP64 update is at its register limit
  uint32_t tl = t;
  asm volatile("" : "+v"(tl));
  const double ms = mass2_of((uint8_t)tl);
  double iu0;
  bool repeat = false;
  for (int it = 0;;) {
    iu0 = m.alpha * rsqrt(ms + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 + m.hu33 * u3 * u3 +
                          2.0 * m.hu13 * u1 * u3);
    const double n1 = g.dt * ((m.hu11 * u1 + m.hu13 * u3) * iu0 - m.beta1);
    const double n2 = g.dt * (m.hu22 * u2 * iu0);
    repeat = n1 == d1 && n2 == d2;
    bool fixed = repeat;
    if (g.iter_tol > 0.0)
      fixed = fixed || fabs(n1 - d1) + fabs(n2 - d2) <= g.iter_tol * (fabs(n1) + fabs(n2));
    d1 = n1;
    d2 = n2;
    if (fixed || ++it >= g.n_iter) break;
    m = coeffs_from(g, rsc_near<SER>(g, tab, i1, x1 + 0.5 * d1, i2, x2 + 0.5 * d2));
  }
  {
    // phi update and the phi velocity at the path midpoint (the J^3 of the
    // deposit); after an exact repeat the last coefficients are already there
    if (!repeat) {
      m = coeffs_from(g, rsc_near<SER>(g, tab, i1, x1 + 0.5 * d1, i2, x2 + 0.5 * d2));
      iu0 = m.alpha * rsqrt(ms + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 + m.hu33 * u3 * u3 +
                            2.0 * m.hu13 * u1 * u3);
    }
    P.phi[k] += g.dt * (m.hu13 * u1 + m.hu33 * u3) * iu0;
    mv.vphi = (m.hu13 * u1 + m.hu33 * u3) * iu0;
  }
  dx1 += d1;
  renormalize(i1, dx1);
  dx2 += d2;
  renormalize(i2, dx2);
  mv.mid = true;
  if (i2 < 0) {
    i2 = 0;
    dx2 = 1.0 - dx2;
    u2 = -u2;
    mv.mid = false;
  } else if (i2 >= g.n_th) {
    i2 = g.n_th - 1;
    dx2 = 1.0 - dx2;
    u2 = -u2;
    mv.mid = false;
  }
  if (i1 < 0 || i1 >= g.n_r) t |= kLeaving;
  // a non-finite or more-than-one-cell move cannot be deposited: drop it
  if (!(fabs(d1) < 1.0 && fabs(d2) < 1.0)) t = kInvalid;
  P.i1[k] = i1;
  P.i2[k] = i2;
  P.dx1[k] = dx1;
  P.dx2[k] = dx2;
  P.u1[k] = u1;
  P.u2[k] = u2;
  P.u3[k] = u3;
  P.tag[k] = t;
  mv.dep = is_live(t) && qm != 0.0;
  mv.ib = i1;
  mv.jb = i2;
  mv.xb = dx1;
  mv.yb = dx2;
  mv.q = (qm * g.charge_scale) * P.w[k];
  mv.u1 = u1;
  mv.u2 = u2;
  mv.u3 = u3;
  mv.cell = cell_key(g, t, i1, i2);
  return mv;
}

// Single-precision form of the same update (see the file comment).
template <int SER, bool kPrev = true>
__device__ inline Move<float> push_one_f32(const Grid& g, const Tables& tab, const GatherPlanesT<float>& fp,
                                           const ParticleArraysT<float>& P, int64_t k) {
  Move<float> mv;
  mv.dep = false;
  mv.cell = g.n_r * g.n_th;
  if (k >= P.n) return mv;
  uint8_t t = P.tag[k];
  if (!is_live(t)) return mv;
  if (t & kLeaving) {
    P.tag[k] = 0;
    return mv;
  }
  int i1 = P.i1[k], i2 = P.i2[k];
  float dx1 = P.dx1[k], dx2 = P.dx2[k];
  if (!in_grid(g, i1, dx1, i2, dx2)) {
    P.tag[k] = kInvalid;
    return mv;
  }
  float u1 = P.u1[k], u2 = P.u2[k], u3 = P.u3[k];
  if (kPrev) {  // the previous position, for a separate deposit
    P.i1p[k] = i1;
    P.i2p[k] = i2;
    P.dx1p[k] = dx1;
    P.dx2p[k] = dx2;
  }
  mv.ia = i1;
  mv.ja = i2;
  mv.xa = dx1;
  mv.ya = dx2;

  FrameT<float> f;
  GradT<float> d;
  if (i1 < g.i_fp64) {
    // horizon region: metric and derivatives in FP64, then rounded
    Frame fd;
    Grad dd;
    frame_from(g, rsc_near<SER>(g, tab, i1, (double)i1 + dx1, i2, (double)i2 + dx2), &fd, &dd);
    f.c = CoeffsT<float>{(float)fd.c.alpha, (float)fd.c.beta1, (float)fd.c.hu11,
                         (float)fd.c.hu22, (float)fd.c.hu33, (float)fd.c.hu13};
    f.s11 = (float)fd.s11;
    f.s22 = (float)fd.s22;
    f.s33 = (float)fd.s33;
    f.k13 = (float)fd.k13;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      d.alpha[q] = (float)dd.alpha[q];
      d.beta1[q] = (float)dd.beta1[q];
      d.hu11[q] = (float)dd.hu11[q];
      d.hu22[q] = (float)dd.hu22[q];
      d.hu33[q] = (float)dd.hu33[q];
      d.hu13[q] = (float)dd.hu13[q];
    }
  } else {
    frame_from(g, rsc_near_f<SER>(g, tab, i1, dx1, i2, dx2), &f, &d);
  }
  const float qm = (float)species_sign(t);
  const float ms = (float)mass2_of(t);
  if (qm != 0.0f) {
    const float D1 = interp<1, 0>(g, fp.D[0], i1, dx1, i2, dx2);
    const float D2 = interp<0, 1>(g, fp.D[1], i1, dx1, i2, dx2);
    const float D3 = interp<0, 0>(g, fp.D[2], i1, dx1, i2, dx2);
    const float B1 = interp<0, 1>(g, fp.B[0], i1, dx1, i2, dx2);
    const float B2 = interp<1, 0>(g, fp.B[1], i1, dx1, i2, dx2);
    const float B3 = interp<1, 1>(g, fp.B[2], i1, dx1, i2, dx2);
    const float al = f.c.alpha, ais11 = al * rcp(f.s11);
    const float E[3] = {ais11 * D1, al * f.s22 * D2, al * f.s33 * (f.k13 * D1 + D3)};
    const float B[3] = {ais11 * B1, al * f.s22 * B2, al * f.s33 * (f.k13 * B1 + B3)};
    const float kb = 0.25f * qm * (float)g.dt;
    em_half(f, E, B, kb, u1, u2, u3);
    geodesic_u(g, f, d, u1, u2, u3, 1.0f);
    em_half(f, E, B, kb, u1, u2, u3);
  } else {
    geodesic_u(g, f, d, u1, u2, u3, ms);  // EM stage skipped for q = 0
  }

  // implicit coordinate update with the displacement (d1, d2) in cells
  const float dt = (float)g.dt;
  float d1 = 0.0f, d2 = 0.0f;
  CoeffsT<float> m = f.c;
  float iu0;
  bool repeat = false;
  for (int it = 0;;) {
    iu0 = m.alpha * rsqrt(ms + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 + m.hu33 * u3 * u3 +
                          2.0f * m.hu13 * u1 * u3);
    const float n1 = dt * ((m.hu11 * u1 + m.hu13 * u3) * iu0 - m.beta1);
    const float n2 = dt * (m.hu22 * u2 * iu0);
    repeat = n1 == d1 && n2 == d2;
    bool fixed = repeat;
    if (g.iter_tol > 0.0)
      fixed = fixed || fabs((double)n1 - (double)d1) + fabs((double)n2 - (double)d2) <=
                           g.iter_tol * (fabs((double)n1) + fabs((double)n2));
    d1 = n1;
    d2 = n2;
    if (fixed || ++it >= g.n_iter) break;
    m = coeffs_from(g, rsc_near_f<SER>(g, tab, i1, dx1 + 0.5f * d1, i2, dx2 + 0.5f * d2));
  }
  {
    if (!repeat) {
      m = coeffs_from(g, rsc_near_f<SER>(g, tab, i1, dx1 + 0.5f * d1, i2, dx2 + 0.5f * d2));
      iu0 = m.alpha * rsqrt(ms + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 + m.hu33 * u3 * u3 +
                            2.0f * m.hu13 * u1 * u3);
    }
    mv.vphi = (m.hu13 * u1 + m.hu33 * u3) * iu0;
    P.phi[k] += dt * mv.vphi;
  }
  dx1 += d1;
  renormalize(i1, dx1);
  dx2 += d2;
  renormalize(i2, dx2);
  mv.mid = true;
  if (i2 < 0) {
    i2 = 0;
    dx2 = 1.0f - dx2;
    u2 = -u2;
    mv.mid = false;
  } else if (i2 >= g.n_th) {
    i2 = g.n_th - 1;
    dx2 = 1.0f - dx2;
    u2 = -u2;
    mv.mid = false;
  }
  if (i1 < 0 || i1 >= g.n_r) t |= kLeaving;
  if (!(fabsf(d1) < 1.0f && fabsf(d2) < 1.0f)) t = kInvalid;
  P.i1[k] = i1;
  P.i2[k] = i2;
  P.dx1[k] = dx1;
  P.dx2[k] = dx2;
  P.u1[k] = u1;
  P.u2[k] = u2;
  P.u3[k] = u3;
  P.tag[k] = t;
  mv.dep = is_live(t) && qm != 0.0f;
  mv.ib = i1;
  mv.jb = i2;
  mv.xb = dx1;
  mv.yb = dx2;
  mv.q = (float)(species_sign(t) * g.charge_scale) * P.w[k];
  mv.u1 = u1;
  mv.u2 = u2;
  mv.u3 = u3;
  mv.cell = cell_key(g, t, i1, i2);
  return mv;
}

// The move of slot k as stored by the push (previous and current position).
template <class T>
__device__ inline Move<T> load_move(const Grid& g, const ParticleArraysT<T>& P, int64_t k) {
  Move<T> mv;
  mv.dep = false;
  mv.mid = false;
  mv.cell = g.n_r * g.n_th;
  if (k >= P.n) return mv;
  const uint8_t t = P.tag[k];
  if (!is_live(t)) return mv;
  const double sg = species_sign(t);
  if (sg == 0.0) return mv;
  mv.dep = true;
  mv.q = (T)(sg * g.charge_scale) * P.w[k];
  mv.ia = P.i1p[k];
  mv.ja = P.i2p[k];
  mv.xa = P.dx1p[k];
  mv.ya = P.dx2p[k];
  mv.ib = P.i1[k];
  mv.jb = P.i2[k];
  mv.xb = P.dx1[k];
  mv.yb = P.dx2[k];
  mv.u1 = P.u1[k];
  mv.u2 = P.u2[k];
  mv.u3 = P.u3[k];
  return mv;
}

template <class T>
struct CurrentPlanesT {
  T* __restrict__ J[3];
};
using CurrentPlanes = CurrentPlanesT<double>;

__device__ inline void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ inline void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

// ------------------------------------------------------------------ deposit
// Charge-conserving zigzag split (Sec. 3.2) of the move from (ia + xa, ja + ya)
// to (ib + xb, jb + yb): the path is cut at the relay point r, each segment
// deposits J^1 and J^2 (normalised by 1/dt) on the edges of the cell it lies
// in, with first-order weights at the segment midpoint; J^3 = q alpha u^3 /
// gamma goes to the four nodes around the path midpoint.
// Particles per block of the deposit passes and the LDS tile of kTI rows x
// dep_tj<T>() columns, measured on the fused pass (blocks of 64, 128 and 256,
// tiles of 6 or 8 rows and 12 to 48 columns): in single precision 64 with
// 8 x 16 (at 4096^2 and 16 per cell -4.5 % against 256 with 8 x 48), in double
// precision 128 with 8 x 16 (at 2048^2 and 90 per cell -2 % against 256 with
// 8 x 48, 64 with 8 x 16 +1 % there; at 512^2 64 and 128 within 2 %); six
// rows often miss a block's footprint (+5 to +13 %)
template <class T>
constexpr int dep_block() { return sizeof(T) == 4 ? 64 : 128; }
template <class T>
constexpr int dep_tj() { return 16; }
constexpr int kTI = 8;
constexpr int kDepRep = 2;  // copies of the deposit tile
// lane-folding levels before the LDS atomics: pairs (measured: quads gave
// nothing in FP64 and, once the FP32 blocks were 64 particles, cost 0.4 % of
// the FP32 fused pass at 4096^2 and 16 per cell)
template <class T>
constexpr int dep_fold() { return 1; }

template <class T>
struct ContribT {
  int ia, ja;         // previous cell: anchor of the 4 x 4 footprint [ia-1, ia+2] x [ja-1, ja+2]
  int di, dj, km, lm; // cell step, J^3 node corner (relative to the anchor)
  T j1[4], j2[4], j3[4];
};

// lapse-weighted phi velocity alpha u^3 / gamma at the path midpoint (ia + xm, ja + ym)
template <int SER>
__device__ inline double vphi_mid(const Grid& g, const Tables& tab, int ia, double xm, int ja,
                                  double ym, double u1, double u2, double u3) {
  const Coeffs m = coeffs_from(g, rsc_near<SER>(g, tab, ia, (double)ia + xm, ja, (double)ja + ym));
  const double iu0 = m.alpha * rsqrt(1.0 + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 + m.hu33 * u3 * u3 +
                                     2.0 * m.hu13 * u1 * u3);
  return (m.hu13 * u1 + m.hu33 * u3) * iu0;
}
template <int SER>
__device__ inline float vphi_mid(const Grid& g, const Tables& tab, int ia, float xm, int ja,
                                 float ym, float u1, float u2, float u3) {
  const CoeffsT<float> m = coeffs_from(g, rsc_near_f<SER>(g, tab, ia, xm, ja, ym));
  const float iu0 = m.alpha * rsqrt(1.0f + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 + m.hu33 * u3 * u3 +
                                    2.0f * m.hu13 * u1 * u3);
  return (m.hu13 * u1 + m.hu33 * u3) * iu0;
}

template <class T, int SER>
__device__ inline bool make_contrib(const Grid& g, const Tables& tab, const Move<T>& mv, ContribT<T>& c) {
  c.ia = c.ja = c.di = c.dj = c.km = c.lm = 0;
  if (!mv.dep) return false;
  const int ia = mv.ia, ja = mv.ja;
  const int di = mv.ib - ia, dj = mv.jb - ja;
  // the zigzag touches at most cells ia-1 .. ia+2: both ends must be in range
  if (!in_grid(g, ia, mv.xa, ja, mv.ya) || !in_deposit_range(g, mv.ib, mv.xb, mv.jb, mv.yb) ||
      abs(di) > 1 || abs(dj) > 1)
    return false;
  const T q = mv.q;
  const T qdt = q / (T)g.dt;
  const T one = (T)1, half = (T)0.5;
  const T xa = mv.xa, ya = mv.ya;
  const T xb = (T)di + mv.xb, yb = (T)dj + mv.yb;
  const T xr = fmin((T)min(0, di) + one, fmax((T)max(0, di), half * (xa + xb)));
  const T yr = fmin((T)min(0, dj) + one, fmax((T)max(0, dj), half * (ya + yb)));
  const T fx1 = qdt * (xr - xa), fy1 = qdt * (yr - ya);
  const T fx2 = qdt * (xb - xr), fy2 = qdt * (yb - yr);
  const T wx1 = half * (xa + xr), wy1 = half * (ya + yr);
  const T wx2 = half * (xr + xb) - (T)di, wy2 = half * (yr + yb) - (T)dj;
  c.ia = ia;
  c.ja = ja;
  c.di = di;
  c.dj = dj;
  // J^1 at (ia, ja), (ia, ja+1), (ib, jb), (ib, jb+1); J^2 at (ia, ja), (ia+1, ja), (ib, jb), (ib+1, jb)
  c.j1[0] = fx1 * (one - wy1);
  c.j1[1] = fx1 * wy1;
  c.j1[2] = fx2 * (one - wy2);
  c.j1[3] = fx2 * wy2;
  c.j2[0] = fy1 * (one - wx1);
  c.j2[1] = fy1 * wx1;
  c.j2[2] = fy2 * (one - wx2);
  c.j2[3] = fy2 * wx2;
  const T xm = half * (xa + xb), ym = half * (ya + yb);
  const T vphi = mv.mid ? mv.vphi : vphi_mid<SER>(g, tab, ia, xm, ja, ym, mv.u1, mv.u2, mv.u3);
  const T fm = floor(xm), gm = floor(ym);
  const T w1 = xm - fm, w2 = ym - gm;
  const T c3 = q * vphi;
  c.km = (int)fm;
  c.lm = (int)gm;
  // J^3 at (km, lm), (km, lm+1), (km+1, lm), (km+1, lm+1)
  c.j3[0] = c3 * (one - w1) * (one - w2);
  c.j3[1] = c3 * (one - w1) * w2;
  c.j3[2] = c3 * w1 * (one - w2);
  c.j3[3] = c3 * w1 * w2;
  // The particle's mirror image in the nearer axis (Sec. 3.3.2) adds the same
  // contribution on an axis node row (j = 0 or n_th) with the component's axis
  // parity: J^1 (even) doubles there, J^3 (odd) cancels, so the axis rows hold
  // the two-sided values the polar-cap update takes with 2 pi.  The footprint
  // spans node rows ja - 1 .. ja + 2, so only particles within two rows of an
  // axis can reach one (a wavefront-uniform skip for cell-sorted particles).
  if (ja <= 1 || ja >= g.n_th - 2) {
    auto e1 = [&](int j) { return (j == 0 || j == g.n_th) ? (T)2 : one; };
    auto e3 = [&](int j) { return (j == 0 || j == g.n_th) ? (T)0 : one; };
    c.j1[0] *= e1(ja);
    c.j1[1] *= e1(ja + 1);
    c.j1[2] *= e1(ja + dj);
    c.j1[3] *= e1(ja + dj + 1);
    const T f0 = e3(ja + c.lm), f1 = e3(ja + c.lm + 1);
    c.j3[0] *= f0;
    c.j3[1] *= f1;
    c.j3[2] *= f0;
    c.j3[3] *= f1;
  }
  return true;
}

// Runs of equal keys in consecutive lanes of a wavefront: `end` is the last
// lane of this lane's run, `head` marks the first lane of a run; `longest` is
// the longest run (wave-uniform).
struct Runs {
  int end, longest;
  bool head;
};

__device__ inline Runs runs_of(int key) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  Runs r;
  r.head = lane == 0 || prev != key;
  const unsigned long long heads = __ballot(r.head);
  const unsigned long long after = lane == 63 ? 0ull : (heads >> (lane + 1));
  r.end = after ? lane + __ffsll((long long)after) - 1 : 63;
  // longest gap between consecutive heads (bit 0 is always set)
  unsigned long long m = heads & ~1ull;
  int last = 0, best = 0;
  while (m) {
    const int b = __ffsll((long long)m) - 1;
    best = max(best, b - last);
    last = b;
    m &= m - 1;
  }
  r.longest = max(best, 64 - last);
  return r;
}

// Sum of v over this lane's run from this lane to the run's end (the head
// ends up with the run total): segmented suffix sum by doubling.
template <class T>
__device__ inline T run_sum(T v, const Runs& r) {
  const int lane = threadIdx.x & 63;
  for (int off = 1; off < r.longest; off <<= 1) {
    const T o = __shfl_down(v, off, 64);
    if (lane + off <= r.end) v += o;
  }
  return v;
}

// Adds the contributions of the lanes of a wavefront through add(comp, i, j,
// value) (absolute node indices), for blocks whose footprint does not fit the
// LDS tile (the values then go straight to the planes as global atomics).
// Particles are cell-sorted, so lanes share cells: the contributions of a run
// of lanes with the same cell are summed across lanes first and the run's
// first lane adds them (global atomics from many lanes on one address would
// serialise).  Every lane of the wavefront must call this (inactive lanes
// with act = false).
template <class T, class Add>
__device__ inline void add_runs(const Grid& g, bool act, const ContribT<T>& c, Add add) {
  const T z = (T)0;
  // segment 1 (previous cell), with segment 2 folded in when the particle stays in its cell
  const bool stay = act && c.di == 0 && c.dj == 0;
  const Runs sa = runs_of(act ? (c.ia + 2) * g.ld + (c.ja + 2) : -1);
  const T a0 = run_sum(act ? c.j1[0] + (stay ? c.j1[2] : z) : z, sa);
  const T a1 = run_sum(act ? c.j1[1] + (stay ? c.j1[3] : z) : z, sa);
  const T a2 = run_sum(act ? c.j2[0] + (stay ? c.j2[2] : z) : z, sa);
  const T a3 = run_sum(act ? c.j2[1] + (stay ? c.j2[3] : z) : z, sa);
  // J^3 nodes around the path midpoint
  const int km = c.ia + c.km, lm = c.ja + c.lm;
  const Runs sm = runs_of(act ? (km + 2) * g.ld + (lm + 2) : -1);
  const T m0 = run_sum(act ? c.j3[0] : z, sm);
  const T m1 = run_sum(act ? c.j3[1] : z, sm);
  const T m2 = run_sum(act ? c.j3[2] : z, sm);
  const T m3 = run_sum(act ? c.j3[3] : z, sm);
  if (act && sa.head) {
    add(0, c.ia, c.ja, a0);
    add(0, c.ia, c.ja + 1, a1);
    add(1, c.ia, c.ja, a2);
    add(1, c.ia + 1, c.ja, a3);
  }
  if (act && !stay) {  // segment 2 in the new cell
    const int ib = c.ia + c.di, jb = c.ja + c.dj;
    add(0, ib, jb, c.j1[2]);
    add(0, ib, jb + 1, c.j1[3]);
    add(1, ib, jb, c.j2[2]);
    add(1, ib + 1, jb, c.j2[3]);
  }
  if (act && sm.head) {
    add(2, km, lm, m0);
    add(2, km, lm + 1, m1);
    add(2, km + 1, lm, m2);
    add(2, km + 1, lm + 1, m3);
  }
}

// Lane exchange inside aligned groups by DPP quad permutation (a VALU move, no
// LDS traffic): level 1 swaps lanes 2k <-> 2k+1, level 2 swaps the pairs of a
// quad (4k, 4k+1 <-> 4k+2, 4k+3).  Every lane of the wavefront must execute it.
template <int L>
__device__ inline int lane_swap(int v) {
  return __builtin_amdgcn_update_dpp(0, v, L == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
template <int L>
__device__ inline float lane_swap(float v) {
  return __int_as_float(lane_swap<L>(__float_as_int(v)));
}
template <int L>
__device__ inline double lane_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_swap<L>((int)(b & 0xffffffffll)), hi = lane_swap<L>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// Adds the contributions of each lane through add(comp, i, j, value) (absolute
// node indices; a particle that stays in its cell folds its second segment into
// the first), with the segment-1 and J^3 values of neighbouring lanes that
// share the same nodes summed first (kFold levels: pairs, then quads): the first lane
// of a folded group adds the group's sum, the others skip those adds.  Cell-
// sorted particles put runs of one cell in consecutive lanes, so this divides
// the LDS atomics on one address by up to 2^kFold.  Every lane of the
// wavefront must call this (inactive lanes with act = false).
template <class T, int kFold, class Add>
__device__ inline void add_lane_folded(const Grid& g, bool act, const ContribT<T>& c, Add add) {
  const int lane = threadIdx.x & 63;
  const T z = (T)0;
  const bool stay = act && c.di == 0 && c.dj == 0;
  const int km = c.ia + c.km, lm = c.ja + c.lm;
  T a[4] = {act ? c.j1[0] + (stay ? c.j1[2] : z) : z, act ? c.j1[1] + (stay ? c.j1[3] : z) : z,
            act ? c.j2[0] + (stay ? c.j2[2] : z) : z, act ? c.j2[1] + (stay ? c.j2[3] : z) : z};
  T m[4] = {act ? c.j3[0] : z, act ? c.j3[1] : z, act ? c.j3[2] : z, act ? c.j3[3] : z};
  const int ka = act ? (c.ia + 2) * g.ld + (c.ja + 2) : -1;
  const int kb = act ? (km + 2) * g.ld + (lm + 2) : -1;
  bool own_a = act, own_m = act;
  bool fa = false, fm = false;  // this lane's pair folded
  if (kFold >= 1) {
    const bool first = (lane & 1) == 0;
    fa = ka >= 0 && lane_swap<1>(ka) == ka;
    fm = kb >= 0 && lane_swap<1>(kb) == kb;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T oa = lane_swap<1>(a[q]), om = lane_swap<1>(m[q]);
      if (fa && first) a[q] += oa;
      if (fm && first) m[q] += om;
    }
    if (fa && !first) own_a = false;
    if (fm && !first) own_m = false;
  }
  if (kFold >= 2) {
    const bool first = (lane & 2) == 0;
    const bool qa = fa && lane_swap<2>((int)fa) != 0 && lane_swap<2>(ka) == ka;
    const bool qm = fm && lane_swap<2>((int)fm) != 0 && lane_swap<2>(kb) == kb;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T oa = lane_swap<2>(a[q]), om = lane_swap<2>(m[q]);
      if (qa && first) a[q] += oa;
      if (qm && first) m[q] += om;
    }
    if (qa && !first) own_a = false;
    if (qm && !first) own_m = false;
  }
  if (own_a) {
    add(0, c.ia, c.ja, a[0]);
    add(0, c.ia, c.ja + 1, a[1]);
    add(1, c.ia, c.ja, a[2]);
    add(1, c.ia + 1, c.ja, a[3]);
  }
  if (act && !stay) {
    const int ib = c.ia + c.di, jb = c.ja + c.dj;
    add(0, ib, jb, c.j1[2]);
    add(0, ib, jb + 1, c.j1[3]);
    add(1, ib, jb, c.j2[2]);
    add(1, ib + 1, jb, c.j2[3]);
  }
  if (own_m) {
    add(2, km, lm, m[0]);
    add(2, km, lm + 1, m[1]);
    add(2, km + 1, lm, m[2]);
    add(2, km + 1, lm + 1, m[3]);
  }
}

// Block-level deposit: the lanes add their contributions (12 values, 8 when a
// particle stays in its cell; neighbouring lanes on the same nodes folded
// first) to an LDS tile over the block's footprint with LDS atomics, then the
// tile rows the footprint covers are added to the planes with one global
// atomic per touched node.  A block whose footprint does not
// fit the tile (its cells wrap from the end of one theta row to the next, or
// its particles have spread) adds wavefront run sums straight to the planes.
// Every lane of the block must call this; on every path it passes a block
// barrier before returning.
template <class T>
__device__ inline void deposit_block(const Grid& g, const CurrentPlanesT<T>& cp, bool act,
                                     const ContribT<T>& c) {
  // kRep copies of the tile: the adding lanes alternate between copies, which
  // divides the same-address conflicts of a cell's run of lanes by kRep
  constexpr int kRep = kDepRep;
  constexpr int kBlk = dep_block<T>(), kTJ = dep_tj<T>();
  __shared__ __align__(16) T tile[kRep][3][kTI][kTJ];
  __shared__ int bound[4][kBlk / 64];
  // block footprint: union of [ia-1, ia+2] x [ja-1, ja+2]
  int v[4] = {act ? c.ia - 1 : INT_MAX, act ? -(c.ia + 2) : INT_MAX, act ? c.ja - 1 : INT_MAX,
              act ? -(c.ja + 2) : INT_MAX};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = __reduce_min_sync(~0ull, v[q]);  // wavefront minimum
    if (lane == 0) bound[q][wv] = m;
  }
  // zero the tile (16-byte stores) while the bounds settle
  {
    constexpr int kVec = 16 / sizeof(T);
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    V* fv = reinterpret_cast<V*>(&tile[0][0][0][0]);
    for (int e = threadIdx.x; e < kRep * 3 * kTI * kTJ / kVec; e += kBlk) fv[e] = V{};
  }
  __syncthreads();
  int b[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    b[q] = bound[q][0];
    for (int w = 1; w < kBlk / 64; ++w) b[q] = min(b[q], bound[q][w]);
  }
  const int i0 = b[0], i1 = -b[1], j0 = b[2], j1 = -b[3];
  if (i0 == INT_MAX) return;  // no live charged particle in this block (uniform)
  const bool fits = (i1 - i0 < kTI) && (j1 - j0 < kTJ);
  if (!fits) {
    add_runs(g, act, c, [&](int comp, int i, int j, T val) { atomic_add(cp.J[comp] + ix(g, i, j), val); });
    return;
  }
  const int rep = (lane >> dep_fold<T>()) % kRep;
  add_lane_folded<T, dep_fold<T>()>(g, act, c,
                               [&](int comp, int i, int j, T val) { atomicAdd(&tile[rep][comp][i - i0][j - j0], val); });
  __syncthreads();
  // flush the footprint rows only, the copies summed in a fixed order
  const int rows = (i1 - i0 + 1) * kTJ;
#pragma unroll
  for (int comp = 0; comp < 3; ++comp) {
    for (int e = threadIdx.x; e < rows; e += kBlk) {
      T val = (&tile[0][comp][0][0])[e];
#pragma unroll
      for (int r = 1; r < kRep; ++r) val += (&tile[r][comp][0][0])[e];
      if (val != (T)0) atomic_add(cp.J[comp] + ix(g, i0 + e / kTJ, j0 + e % kTJ), val);
    }
  }
}

// ------------------------------------------------------------------ cell ranks
// The counting sort by cell (cell_key) needs each live slot's rank among the
// slots of its cell and each cell's count.  A block counts its slots per cell
// in an LDS hash table of 2^kBits cells (open addressing, linear probing; at
// most 2^(kBits-1) slots per block, so a free cell is always found): a slot's
// rank inside the block is its cell's count when it was added.  Then one
// returning atomic per cell present in the block claims the block's ranks of
// that cell on the cell's global counter, and every slot takes its cell's
// base plus its rank inside the block.  Slots with key n_cells claim nothing.
template <int kBits>
struct RankTable {
  int key[1 << kBits];
  int n[1 << kBits];  // count in the block, then the cell's base
};

// The block's table (one LDS object per block, whichever function asks).
template <int kBits>
__device__ inline RankTable<kBits>& block_rank_table() {
  __shared__ RankTable<kBits> rt;
  return rt;
}

template <int kBits>
__device__ inline void rank_clear(RankTable<kBits>& rt) {
  for (int e = (int)threadIdx.x; e < (1 << kBits); e += (int)blockDim.x) {
    rt.key[e] = -1;
    rt.n[e] = 0;
  }
}

// Adds a slot of cell `key` (< n_cells) to the table; returns its entry, and
// in `local` the number of the block's slots of that cell added before it.
template <int kBits>
__device__ inline int rank_insert(RankTable<kBits>& rt, int key, int& local) {
  int h = (int)(((uint32_t)key * 0x9E3779B1u) >> (32 - kBits));  // multiplicative hash
  for (;;) {
    const int old = atomicCAS(&rt.key[h], -1, key);
    if (old == -1 || old == key) break;
    h = (h + 1) & ((1 << kBits) - 1);
  }
  local = atomicAdd(&rt.n[h], 1);
  return h;
}

// The claims: afterwards rt.n holds each present cell's base.  Every thread
// of the block calls this after a barrier that follows the last insert (all
// of a thread's claims are in flight before the first is waited for).
template <int kBits, int kThreads>
__device__ inline void rank_claim(RankTable<kBits>& rt, int* __restrict__ counts) {
  constexpr int kE = (1 << kBits) / kThreads;
  int base[kE];
#pragma unroll
  for (int e = 0; e < kE; ++e) {
    const int h = e * kThreads + (int)threadIdx.x;
    const int key = rt.key[h];
    base[e] = key >= 0 ? atomicAdd(counts + key, rt.n[h]) : 0;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kE; ++e) rt.n[e * kThreads + (int)threadIdx.x] = base[e];
  __syncthreads();
}

// Table bits for the dep_block<T>() slots of a fused block: twice as many
// cells as slots.
template <class T>
constexpr int push_rank_bits() { return sizeof(T) == 4 ? 7 : 8; }
static_assert((1 << (push_rank_bits<float>() - 1)) >= dep_block<float>(), "rank table too small");
static_assert((1 << (push_rank_bits<double>() - 1)) >= dep_block<double>(), "rank table too small");

// The rank pass of the sort inside a fused push + deposit block: slot k's key
// after the push is `cell`; its rank goes to i1p (the previous position is not
// stored by the fused pass).  The table was cleared at the start of the
// kernel and a block barrier (the deposit's) has passed since.
template <class T>
__device__ inline void rank_fused(const Grid& g, int* __restrict__ i1p, int64_t k, int cell,
                                  int* __restrict__ counts) {
  constexpr int kBits = push_rank_bits<T>();
  RankTable<kBits>& rt = block_rank_table<kBits>();
  int local = 0, entry = -1;
  if (cell < g.n_r * g.n_th) entry = rank_insert(rt, cell, local);
  __syncthreads();
  rank_claim<kBits, dep_block<T>()>(rt, counts);
  if (entry >= 0) i1p[k] = rt.n[entry] + local;
}

// ------------------------------------------------------------------ kernels
// The FP64 push kernels are held to 128 VGPRs (4 wavefronts per SIMD; no
// spills on the series paths): on gfx950 the push is latency- and issue-bound,
// and the fourth wavefront hides more than the compiler's own choice (~160
// VGPRs, 3 wavefronts, a 10-15 % slower pass); a fifth (96 VGPRs) spills
// 148 B per lane and runs about 30 % slower.
#define GRPIC_FP64_PUSH_OCCUPANCY __attribute__((amdgpu_waves_per_eu(4)))

template <int SER>
__global__ void __launch_bounds__(256) GRPIC_FP64_PUSH_OCCUPANCY
push_kernel(Grid g, Tables tab, GatherPlanesT<double> fp, ParticleArrays P) {
  (void)push_one<SER>(g, tab, fp, P, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

template <int SER>
__global__ void __launch_bounds__(256) push_kernel_f32(Grid g, Tables tab, GatherPlanesT<float> fp,
                                                       ParticleArraysT<float> P) {
  (void)push_one_f32<SER>(g, tab, fp, P, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

template <class T, int SER>
__global__ void __launch_bounds__(dep_block<T>()) deposit_kernel(Grid g, Tables tab, ParticleArraysT<T> P,
                                                            CurrentPlanesT<T> cp) {
  const Move<T> mv = load_move(g, P, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  ContribT<T> c;
  const bool act = make_contrib<T, SER>(g, tab, mv, c);
  deposit_block(g, cp, act, c);
}

// Push and deposit in one pass: the deposit takes the move from registers and
// J^3 from the push's own midpoint metric; the previous position is not
// stored.  kRank: the pass also ranks the slots by their cell after the push
// for the cell sort (rank_fused; counts: the sort's zeroed cell counters).
template <int SER, bool kRank>
__global__ void __launch_bounds__(dep_block<double>()) GRPIC_FP64_PUSH_OCCUPANCY
push_deposit_kernel(Grid g, Tables tab, GatherPlanesT<double> fp, ParticleArrays P, CurrentPlanes cp, int* counts) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (kRank) rank_clear(block_rank_table<push_rank_bits<double>()>());
  const Move<double> mv = push_one<SER, false>(g, tab, fp, P, k);
  ContribT<double> c;
  const bool act = make_contrib<double, SER>(g, tab, mv, c);
  deposit_block(g, cp, act, c);
  if constexpr (kRank) rank_fused<decltype(mv.u1)>(g, P.i1p, k, mv.cell, counts);
}

// library path in FP64 (coarse grids and the general quasi-spherical map):
// the library exp and sincos and the map factors need more registers than the
// series paths; three wavefronts per SIMD leave room for them without spills
template <bool kRank>
__global__ void __launch_bounds__(dep_block<double>()) __attribute__((amdgpu_waves_per_eu(3)))
push_deposit_kernel_lib(Grid g, Tables tab, GatherPlanesT<double> fp, ParticleArrays P, CurrentPlanes cp,
                        int* counts) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (kRank) rank_clear(block_rank_table<push_rank_bits<double>()>());
  const Move<double> mv = push_one<0, false>(g, tab, fp, P, k);
  ContribT<double> c;
  const bool act = make_contrib<double, 0>(g, tab, mv, c);
  deposit_block(g, cp, act, c);
  if constexpr (kRank) rank_fused<decltype(mv.u1)>(g, P.i1p, k, mv.cell, counts);
}

template <int SER, bool kRank>
__device__ inline void push_deposit_f32(const Grid& g, const Tables& tab, const GatherPlanesT<float>& fp,
                                        const ParticleArraysT<float>& P, const CurrentPlanesT<float>& cp,
                                        int* counts) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (kRank) rank_clear(block_rank_table<push_rank_bits<float>()>());
  const Move<float> mv = push_one_f32<SER, false>(g, tab, fp, P, k);
  ContribT<float> c;
  const bool act = make_contrib<float, SER>(g, tab, mv, c);
  deposit_block(g, cp, act, c);
  if constexpr (kRank) rank_fused<decltype(mv.u1)>(g, P.i1p, k, mv.cell, counts);
}

// series paths: 5 wavefronts per SIMD (96 VGPRs: the compiler's own
// allocation without the rank pass; the rank pass would take it past 96)
template <int SER, bool kRank>
__global__ void __launch_bounds__(dep_block<float>()) __attribute__((amdgpu_waves_per_eu(5))) push_deposit_kernel_f32(Grid g, Tables tab, GatherPlanesT<float> fp,
                                                                     ParticleArraysT<float> P,
                                                                     CurrentPlanesT<float> cp, int* counts) {
  push_deposit_f32<SER, kRank>(g, tab, fp, P, cp, counts);
}

// library path (coarse grids and the general quasi-spherical map): held to 5
// wavefronts per SIMD (a few spilled registers), 11 % faster than the 4 that
// its 100 VGPRs would give
template <bool kRank>
__global__ void __launch_bounds__(dep_block<float>()) __attribute__((amdgpu_waves_per_eu(5)))
push_deposit_kernel_f32_lib(Grid g, Tables tab, GatherPlanesT<float> fp, ParticleArraysT<float> P,
                            CurrentPlanesT<float> cp, int* counts) {
  push_deposit_f32<0, kRank>(g, tab, fp, P, cp, counts);
}

}  // namespace grpic
