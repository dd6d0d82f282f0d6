// geometry.hpp -- grid description and Kerr-Schild 3+1 geometry in code
// coordinates, evaluated on the device (and on the host for dt and tables).
//
// Code coordinates (App. A, quasi-spherical Kerr-Schild): r = r0 + exp(xi),
//   xi = xi_min + x1 dxi; theta = eta + 2 h0 eta (pi - 2 eta)(pi - eta) / pi^2,
//   eta = x2 dth (dth is the uniform eta spacing); phi with dphi = 1.
//   r0 = h0 = 0 is the logarithmic-r, uniform-theta grid.
// Kerr-Schild 3+1 split (Sec. 2.1, App. A), with S2 = Sigma + 2 M r:
//   Sigma = r^2 + a^2 cos^2, Delta = r^2 - 2 M r + a^2,
//   A = (r^2 + a^2)^2 - a^2 Delta sin^2, alpha^2 = Sigma / S2,
//   beta^r = 2 M r / S2, h^rr = A / (Sigma S2), h^rphi = a / Sigma,
//   h^thth = 1 / Sigma, h^phiphi = 1 / (Sigma sin^2),
//   h_rr = S2 / Sigma, h_rphi = -a (S2 / Sigma) sin^2, h_thth = Sigma,
//   h_phiphi = A sin^2 / Sigma, sqrt(h) = Sigma sin / alpha.
// A covariant index 1 carries a factor R = dr/dx1 = dxi (r - r0), index 2 a
// factor T = dtheta/dx2; contravariant indices the inverse factors.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace grpic {

constexpr double kPi = 3.14159265358979323846;

// Everything a kernel needs to know about the grid and the run, by value.
struct Grid {
  double a, M;
  double xi_min, dxi, dth, inv_dth2;  // xi_min = log(r_min - r0); dth: eta spacing
  double r0, h0;                      // quasi-spherical map (0, 0: log r, uniform theta)
  double dt;
  double small_angle;
  double charge_scale;
  double iter_tol;  // relative FP64 convergence test of the implicit iterations (0: off)
  // sin, cos of the clamped polar angles small_angle and pi - small_angle
  double sin_lo, cos_lo, sin_hi, cos_hi;
  int n_r, n_th, ng, ld;  // ld = n_th + 2 ng (row length of a plane)
  int n_iter, n_filter, n_absorb;
  int ser;                // series used by the push for in-cell offsets (0 = library)
  double axis_band;       // short series: polar band next to each axis (4 cells)
  // uniform values the push would otherwise form per wavefront in vector
  // registers: a^2, 2 M, pi - small_angle, pi - axis_band
  double a2, two_M, th_hi, band_hi;
  int i_fp64;             // single-precision push: cells i1 < i_fp64 (r < 3 M, the
                          // horizon region) take the metric and its derivatives in FP64
  int64_t plane;          // reals per plane
};

__host__ __device__ inline int64_t ix(const Grid& g, int i, int j) {
  return (int64_t)(i + g.ng) * g.ld + (j + g.ng);
}

// 1-D coordinate tables, indexed by (index + ng); [0] integer, [1] half-integer
// points: r and 1/(R deta) along x1 (R = dr/dx1, deta the eta spacing); sin,
// cos, 1/sin (0 on the axis), T = dtheta/dx2 and deta/T along x2 (T = deta and
// deta/T = 1 when h0 = 0).  rf: r - r0 at integer x1, sf, cf: sin, cos at
// integer x2, in single precision.
struct Tables {
  const double* __restrict__ r[2];
  const double* __restrict__ ird[2];
  const double* __restrict__ s[2];
  const double* __restrict__ c[2];
  const double* __restrict__ is[2];
  const double* __restrict__ td[2];
  const double* __restrict__ eta_t[2];
  const float* __restrict__ rf;
  const float* __restrict__ sf;
  const float* __restrict__ cf;
};

// Pusher coefficients at a point: lapse, shift and inverse spatial metric.
template <class R>
struct CoeffsT {
  R alpha, beta1, hu11, hu22, hu33, hu13;
};

// Coefficients plus the tetrad factors of App. A at a point:
// s11 = sqrt(h^11), s22 = sqrt(h_22), s33 = sqrt(h_33), k13 = h_13 / h_33.
template <class R>
struct FrameT {
  CoeffsT<R> c;
  R s11, s22, s33, k13;
};

// d/dx1 ([0]) and d/dx2 ([1]) of the pusher coefficients.
template <class R>
struct GradT {
  R alpha[2], beta1[2], hu11[2], hu22[2], hu33[2], hu13[2];
};

// r, sin(theta), cos(theta) of a point, and the map factors there:
// rd = dr/dx1, td = dtheta/dx2, itd2 = 1/td^2, dtd = d td / dx2
template <class R>
struct RSCT {
  R r, s, c;
  R rd, td, itd2, dtd;
};

using Coeffs = CoeffsT<double>;
using Frame = FrameT<double>;
using Grad = GradT<double>;
using RSC = RSCT<double>;

__host__ __device__ inline double clamp_theta(const Grid& g, double th) {
  return fmin(fmax(th, g.small_angle), kPi - g.small_angle);
}

__host__ __device__ inline void sin_cos(double th, double* s, double* c) {
#ifdef __HIP_DEVICE_COMPILE__
  sincos(th, s, c);
#else
  *s = std::sin(th);
  *c = std::cos(th);
#endif
}

// 1/x and 1/sqrt(x) for positive normal x: hardware seeds refined by Newton
// steps on the device (two in double, one in single; error ~1 ulp), plain
// division on the host.
__host__ __device__ inline double rcp(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
#else
  return 1.0 / x;
#endif
}

__host__ __device__ inline double rsqrt(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
#else
  return 1.0 / std::sqrt(x);
#endif
}

__host__ __device__ inline float rcp(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  const float y = __builtin_amdgcn_rcpf(x);
  return fmaf(y, fmaf(-x, y, 1.0f), y);
#else
  return 1.0f / x;
#endif
}

__host__ __device__ inline float rsqrt(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  const float y = __builtin_amdgcn_rsqf(x);
  return fmaf(y, fmaf(-0.5f * x * y, y, 0.5f), y);
#else
  return 1.0f / std::sqrt(x);
#endif
}

// The quasi-spherical map (App. A): r and R = dr/dx1 at x1; theta,
// T = dtheta/dx2 and dT/dx2 at x2.  Beyond either axis the polar map is
// continued by reflection (theta(-x2) = -theta(x2), theta(2 n_th - x2) =
// 2 pi - theta(x2)), so that geometry there mirrors the interior.
__host__ __device__ inline void map_r(const Grid& g, double x1, double* r, double* rd) {
  const double e = exp(g.xi_min + x1 * g.dxi);
  *r = g.r0 + e;
  *rd = g.dxi * e;
}

__host__ __device__ inline void map_theta(const Grid& g, double x2, double* th, double* td,
                                          double* dtd) {
#pragma clang fp contract(off)
  double sg = 1.0, off = 0.0;
  if (x2 < 0.0) {
    x2 = -x2;
    sg = -1.0;
  } else if (x2 > (double)g.n_th) {
    x2 = 2.0 * g.n_th - x2;
    sg = -1.0;
    off = 2.0 * kPi;
  }
  // theta is rounded from exactly these operations in this order (no fused
  // multiply-adds, a true division by pi^2): next to theta = pi one unit in
  // its last place is a relative 1e-13 of sin(theta) a few 1e-4 rad from the
  // axis, so every evaluation of the map must round alike
  const double eta = x2 * g.dth, y = eta * (1.0 / kPi), h0 = g.h0;
  *th = off + sg * (eta + 2.0 * h0 * eta * (kPi - 2.0 * eta) * (kPi - eta) / (kPi * kPi));
  *td = g.dth * (1.0 + 2.0 * h0 + 12.0 * h0 * y * (y - 1.0));
  *dtd = sg * g.dth * g.dth * 12.0 * h0 * (2.0 * y - 1.0) * (1.0 / kPi);
}

// r, clamped sin/cos and the map factors by the library functions
__host__ __device__ inline RSC rsc_direct(const Grid& g, double x1, double x2) {
  RSC p;
  map_r(g, x1, &p.r, &p.rd);
  double th;
  map_theta(g, x2, &th, &p.td, &p.dtd);
  const double it = rcp(p.td);
  p.itd2 = it * it;
  sin_cos(clamp_theta(g, th), &p.s, &p.c);
  return p;
}

// Inverse metric, lapse and shift at a point (R = dr/dx1).
template <class R>
__host__ __device__ inline CoeffsT<R> coeffs_from(const Grid& g, RSCT<R> p) {
  const R r = p.r, s = p.s, c = p.c;
  // (FP64: a^2 and 2 M from the grid, held in scalar registers; the
  // single-precision form keeps forming them, which suits its allocation)
  const R a = (R)g.a, a2 = sizeof(R) == 8 ? (R)g.a2 : a * a, r2 = r * r;
  const R tMr = (sizeof(R) == 8 ? (R)g.two_M : (R)(2.0 * g.M)) * r;
  const R Sig = r2 + a2 * c * c;
  const R S2 = Sig + tMr;
  const R ra = r2 + a2;
  const R s2 = s * s;
  const R A = ra * ra - a2 * (ra - tMr) * s2;
  const R Rr = p.rd;
  // one reciprocal for 1/Sigma, 1/S2, 1/sin^2 and 1/R
  const R q = rcp(Sig * S2 * s2 * Rr);
  const R iSig = S2 * s2 * Rr * q, iS2 = Sig * s2 * Rr * q;
  const R is2 = Sig * S2 * Rr * q, iR = Sig * S2 * s2 * q;
  CoeffsT<R> m;
  const R y = Sig * iS2;
  m.alpha = y * rsqrt(y);
  m.beta1 = tMr * iS2 * iR;
  m.hu11 = A * iSig * iS2 * iR * iR;
  m.hu13 = a * iSig * iR;
  m.hu22 = iSig * p.itd2;
  m.hu33 = iSig * is2;
  return m;
}

__host__ __device__ inline Coeffs coeffs_at(const Grid& g, double x1, double x2) {
  return coeffs_from(g, rsc_direct(g, x1, x2));
}

// Coefficients, tetrad factors and first derivatives at a point.
template <class R>
__host__ __device__ inline void frame_from(const Grid& g, RSCT<R> p, FrameT<R>* f, GradT<R>* d) {
  const R r = p.r, s = p.s, c = p.c;
  const R a = (R)g.a, M = (R)g.M, dxi = (R)g.dxi, dth = p.td;
  const R a2 = sizeof(R) == 8 ? (R)g.a2 : a * a, r2 = r * r;
  const R tMr = sizeof(R) == 8 ? (R)g.two_M * r : (R)2 * M * r;
  const R Sig = r2 + a2 * c * c;
  const R S2 = Sig + tMr;
  const R ra = r2 + a2;
  const R Del = ra - tMr;
  const R s2 = s * s;
  const R A = ra * ra - a2 * Del * s2;
  const R Rr = p.rd;
  const R q = rcp(Sig * S2 * s2 * Rr * A);
  const R iSig = S2 * s2 * Rr * A * q, iS2 = Sig * s2 * Rr * A * q;
  const R is2 = Sig * S2 * Rr * A * q, iR = Sig * S2 * s2 * A * q;
  const R iA = Sig * S2 * s2 * Rr * q;
  const R y = Sig * iS2;
  const R ialpha = rsqrt(y);
  const R alpha = y * ialpha;

  f->c.alpha = alpha;
  f->c.beta1 = tMr * iS2 * iR;
  const R hrr = A * iSig * iS2;
  f->c.hu11 = hrr * iR * iR;
  f->c.hu13 = a * iSig * iR;
  f->c.hu22 = iSig * p.itd2;
  f->c.hu33 = iSig * is2;
  f->s11 = hrr * rsqrt(hrr) * iR;
  f->s22 = Sig * rsqrt(Sig) * dth;
  const R AiS = A * iSig;
  f->s33 = AiS * rsqrt(AiS) * s;
  f->k13 = -a * Rr * S2 * iA;

  // radial and polar derivatives of Sigma, A (S2 shares dSigma/dtheta)
  const R dSig_r = (R)2 * r, dSig_t = (R)-2 * a2 * s * c;
  const R dA_r = (R)4 * r * ra - a2 * s2 * ((R)2 * r - (R)2 * M);
  const R dA_t = (R)-2 * a2 * Del * s * c;
  const R iS22 = iS2 * iS2, iSig2 = iSig * iSig;

  // alpha
  d->alpha[0] = Rr * M * ((R)2 * r2 - Sig) * ialpha * iS22;
  d->alpha[1] = dth * M * r * dSig_t * ialpha * iS22;
  // beta^1 = beta^r / R
  const R dbr_r = (R)2 * M * (Sig - (R)2 * r2) * iS22;
  const R dbr_t = -tMr * dSig_t * iS22;
  d->beta1[0] = dbr_r - dxi * f->c.beta1;
  d->beta1[1] = dth * dbr_t * iR;
  // h^11 = h^rr / R^2
  const R dhrr_r = (dA_r - hrr * (dSig_r * S2 + Sig * (dSig_r + (R)2 * M))) * iSig * iS2;
  const R dhrr_t = (dA_t - hrr * (R)2 * dSig_t * (Sig + M * r)) * iSig * iS2;
  d->hu11[0] = dhrr_r * iR - (R)2 * dxi * f->c.hu11;
  d->hu11[1] = dth * dhrr_t * iR * iR;
  // h^13 = a / (Sigma R)
  d->hu13[0] = -a * dSig_r * iSig2 - dxi * f->c.hu13;
  d->hu13[1] = -dth * a * dSig_t * iSig2 * iR;
  // h^22 = 1 / (Sigma T^2), T = dtheta/dx2 (its own x2 derivative included)
  d->hu22[0] = -Rr * dSig_r * iSig2 * p.itd2;
  d->hu22[1] = -(dth * dSig_t * iSig2 + (R)2 * p.dtd * iSig * dth * p.itd2) * p.itd2;
  // h^33 = 1 / (Sigma sin^2)
  d->hu33[0] = -Rr * dSig_r * iSig2 * is2;
  d->hu33[1] = -dth * (dSig_t + (R)2 * Sig * c * s * is2) * iSig2 * is2;
}

__host__ __device__ inline void frame_at(const Grid& g, double x1, double x2, Frame* f, Grad* d) {
  frame_from(g, rsc_direct(g, x1, x2), f, d);
}

// Geometry at a grid location for the field solver (theta not clamped).
struct Cell {
  double alpha, beta1, hl11, hl22, hl33, hl13;
  double sqrt_h, sqrt_ht;  // sqrt(h) and sqrt(h) / sin(theta)
};

__host__ __device__ inline Cell cell_at(const Grid& g, double x1, double x2) {
  double r, R, th, T, dT;
  map_r(g, x1, &r, &R);
  map_theta(g, x2, &th, &T, &dT);
  double s, c;
  sin_cos(th, &s, &c);
  const double a2 = g.a * g.a, r2 = r * r, tMr = 2.0 * g.M * r;
  const double Sig = r2 + a2 * c * c;
  const double S2 = Sig + tMr;
  const double ra = r2 + a2;
  const double A = ra * ra - a2 * (ra - tMr) * s * s;
  const double iSig = 1.0 / Sig;
  const double opz = S2 * iSig;  // 1 + z
  Cell e;
  e.alpha = sqrt(Sig / S2);
  e.beta1 = tMr / (S2 * R);
  e.hl11 = opz * R * R;
  e.hl22 = Sig * T * T;
  e.hl33 = A * s * s * iSig;
  e.hl13 = -g.a * opz * s * s * R;
  e.sqrt_ht = R * T * Sig / e.alpha;
  e.sqrt_h = e.sqrt_ht * s;
  return e;
}

// gamma = sqrt(m^2 + h^ij u_i u_j) (Sec. 2.3; mass2 = 1 massive, 0 massless)
__host__ __device__ inline double gamma_of(const Coeffs& m, double u1, double u2, double u3,
                                           double mass2 = 1.0) {
  return sqrt(mass2 + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 + m.hu33 * u3 * u3 +
              2.0 * m.hu13 * u1 * u3);
}

}  // namespace grpic
