// particles.hpp -- push and deposit kernels (FP64 form).
//
// One particle per lane; structure-of-arrays loads and stores are contiguous
// across a wavefront.  The push follows Sec. 3.1 steps 1-11 of the paper; the
// deposit Sec. 3.2.
#pragma once

#include <climits>

#include "geometry.hpp"

namespace grpic {

constexpr uint8_t kLeaving = 0x80;
constexpr uint8_t kInvalid = 0x40;  // dropped by a bounds guard; never used again
constexpr uint8_t kSpecies = 0x03;

__host__ __device__ inline bool is_live(uint8_t t) { return t != 0 && !(t & kInvalid); }

// a position inside the grid (what the push may start from)
__device__ inline bool in_grid(const Grid& g, int i1, double dx1, int i2, double dx2) {
  return i1 >= 0 && i1 < g.n_r && i2 >= 0 && i2 < g.n_th && dx1 >= 0.0 && dx1 <= 1.0 &&
         dx2 >= 0.0 && dx2 <= 1.0;
}

// a position the deposit may write around: one cell beyond the radial edges
__device__ inline bool in_deposit_range(const Grid& g, int i1, double dx1, int i2, double dx2) {
  return i1 >= -1 && i1 <= g.n_r && i2 >= 0 && i2 < g.n_th && dx1 >= 0.0 && dx1 <= 1.0 &&
         dx2 >= 0.0 && dx2 <= 1.0;
}

struct ParticleArrays {
  int32_t* __restrict__ i1;
  int32_t* __restrict__ i2;
  double* __restrict__ dx1;
  double* __restrict__ dx2;
  double* __restrict__ u1;
  double* __restrict__ u2;
  double* __restrict__ u3;
  double* __restrict__ w;
  double* __restrict__ phi;
  int32_t* __restrict__ i1p;
  int32_t* __restrict__ i2p;
  double* __restrict__ dx1p;
  double* __restrict__ dx2p;
  uint8_t* __restrict__ tag;
  int64_t n;
};

struct GatherPlanes {
  const double* __restrict__ D[3];
  const double* __restrict__ B[3];
};

__device__ inline double species_sign(uint8_t t) {
  const int s = t & kSpecies;
  return s == 1 ? 1.0 : (s == 2 ? -1.0 : 0.0);
}

// First-order interpolation in code coordinates of a plane staggered by half a
// cell in x1 (H1) and/or x2 (H2).
template <int H1, int H2>
__device__ inline double interp(const Grid& g, const double* __restrict__ F, int i1, double dx1,
                                int i2, double dx2) {
  int k1 = i1, k2 = i2;
  double w1 = dx1, w2 = dx2;
  if (H1) {
    const bool up = dx1 >= 0.5;
    k1 = up ? i1 : i1 - 1;
    w1 = up ? dx1 - 0.5 : dx1 + 0.5;
  }
  if (H2) {
    const bool up = dx2 >= 0.5;
    k2 = up ? i2 : i2 - 1;
    w2 = up ? dx2 - 0.5 : dx2 + 0.5;
  }
  const double* p = F + ix(g, k1, k2);
  const double f00 = p[0], f01 = p[1], f10 = p[g.ld], f11 = p[g.ld + 1];
  const double a0 = f00 + w2 * (f01 - f00);
  const double a1 = f10 + w2 * (f11 - f10);
  return a0 + w1 * (a1 - a0);
}

// Relativistic Boris rotation for duration tau in an orthonormal frame.
__device__ inline void boris(double& ux, double& uy, double& uz, const double E[3],
                             const double B[3], double k /* = qm tau / 2 */) {
  const double mx = ux + k * E[0], my = uy + k * E[1], mz = uz + k * E[2];
  const double ig = k / sqrt(1.0 + mx * mx + my * my + mz * mz);
  const double tx = B[0] * ig, ty = B[1] * ig, tz = B[2] * ig;
  const double f = 2.0 / (1.0 + tx * tx + ty * ty + tz * tz);
  const double sx = f * tx, sy = f * ty, sz = f * tz;
  const double px = mx + (my * tz - mz * ty);
  const double py = my + (mz * tx - mx * tz);
  const double pz = mz + (mx * ty - my * tx);
  ux = mx + (py * sz - pz * sy) + k * E[0];
  uy = my + (pz * sx - px * sz) + k * E[1];
  uz = mz + (px * sy - py * sx) + k * E[2];
}

// EM half step: covariant -> tetrad (App. A), Boris, tetrad -> covariant.
__device__ inline void em_half(const Frame& f, const double E[3], const double B[3], double k,
                               double& u1, double& u2, double& u3) {
  double x = f.s11 * (u1 - f.k13 * u3);
  double y = u2 / f.s22;
  double z = u3 / f.s33;
  boris(x, y, z, E, B, k);
  u1 = x / f.s11 + f.k13 * f.s33 * z;
  u2 = f.s22 * y;
  u3 = f.s33 * z;
}

// Implicit-midpoint geodesic momentum update at fixed x^n (eq.
// discretized-geodesic-u); u_3 is untouched.
__device__ inline void geodesic_u(const Grid& g, const Frame& f, const Grad& d, double& u1,
                                  double& u2, double u3) {
  const Coeffs& m = f.c;
  const double s1 = u1, s2 = u2;
  const double u33 = u3 * u3;
  double t1 = s1, t2 = s2;
  for (int it = 0; it < g.n_iter; ++it) {
    const double b1 = 0.5 * (s1 + t1), b2 = 0.5 * (s2 + t2);
    const double Q = 1.0 + m.hu11 * b1 * b1 + m.hu22 * b2 * b2 + m.hu33 * u33 +
                     2.0 * m.hu13 * b1 * u3;
    const double ig = rsqrt(Q);
    const double gb = Q * ig;
    const double h = 0.5 * m.alpha * ig;
    double fr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double q = d.hu11[i] * b1 * b1 + d.hu22[i] * b2 * b2 + d.hu33[i] * u33 +
                       2.0 * d.hu13[i] * b1 * u3;
      fr[i] = -gb * d.alpha[i] + b1 * d.beta1[i] - h * q;
    }
    const double n1 = s1 + g.dt * fr[0], n2 = s2 + g.dt * fr[1];
    // exact repeat: the fixed point of the map; or the optional FP64 convergence test
    const bool fixed = (n1 == t1 && n2 == t2) ||
                       fabs(n1 - t1) + fabs(n2 - t2) <= g.iter_tol * (fabs(n1) + fabs(n2));
    t1 = n1;
    t2 = n2;
    if (fixed) break;
  }
  u1 = t1;
  u2 = t2;
}

__device__ inline void renormalize(int& i, double& dx) {
  const double f = floor(dx);
  i += (int)f;
  dx -= f;
  if (dx >= 1.0) {
    dx -= 1.0;
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

// pi - (pi rounded to double)
constexpr double kPiLo = 1.2246467991473531772e-16;

// r, sin, cos at code position (x1, x2) near cell (i1, i2) (|x - i| <= 1.5):
// r = r_i exp((x1 - i1) dxi); the polar angle is first rounded and clamped as
// theta = clamp(x2 dth), and the result is the sine and cosine of that double:
// by the short series on theta itself within 0.11 of theta = 0, on
// psi = pi - theta (exact subtraction plus the low part of pi) within 0.11 of
// theta = pi, so that sin keeps its relative precision next to both axes, and
// by angle addition from the tables elsewhere.  Library functions when the
// grid is too coarse for the short series.
template <bool FAST>
__device__ inline RSC rsc_near(const Grid& g, const Tables& t, int i1, double x1, int i2, double x2) {
  if (!FAST) return rsc_direct(g, x1, x2);
  RSC p;
  p.r = t.r[0][i1 + g.ng] * exp_small((x1 - (double)i1) * g.dxi);
  const double th = x2 * g.dth;
  if (th <= g.small_angle) {
    p.s = g.sin_lo;
    p.c = g.cos_lo;
  } else if (th >= kPi - g.small_angle) {
    p.s = g.sin_hi;
    p.c = g.cos_hi;
  } else if (th <= 0.11) {
    sincos_small(th, &p.s, &p.c);
  } else if (th >= kPi - 0.11) {
    double cq;
    sincos_small((kPi - th) + kPiLo, &p.s, &cq);
    p.c = -cq;
  } else {
    double sp, cp;
    sincos_small(th - (double)i2 * g.dth, &sp, &cp);
    const double sj = t.s[0][i2 + g.ng], cj = t.c[0][i2 + g.ng];
    p.s = fma(sj, cp, cj * sp);
    p.c = fma(cj, cp, -(sj * sp));
  }
  return p;
}

template <bool FAST>
__global__ void __launch_bounds__(256) push_kernel(Grid g, Tables tab, GatherPlanes fp, ParticleArrays P) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  uint8_t t = P.tag[k];
  if (!is_live(t)) return;
  if (t & kLeaving) {
    P.tag[k] = 0;
    return;
  }
  int i1 = P.i1[k], i2 = P.i2[k];
  double dx1 = P.dx1[k], dx2 = P.dx2[k];
  if (!in_grid(g, i1, dx1, i2, dx2)) {  // corrupt input: drop, never index with it
    P.tag[k] = kInvalid;
    return;
  }
  double u1 = P.u1[k], u2 = P.u2[k], u3 = P.u3[k];
  P.i1p[k] = i1;
  P.i2p[k] = i2;
  P.dx1p[k] = dx1;
  P.dx2p[k] = dx2;

  const double x1 = (double)i1 + dx1, x2 = (double)i2 + dx2;
  Frame f;
  Grad d;
  frame_from(g, rsc_near<FAST>(g, tab, i1, x1, i2, x2), &f, &d);
  const double qm = species_sign(t);
  if (qm != 0.0) {
    // D^i, B^i at x^n -> tetrad components, scaled by the lapse
    const double D1 = interp<1, 0>(g, fp.D[0], i1, dx1, i2, dx2);
    const double D2 = interp<0, 1>(g, fp.D[1], i1, dx1, i2, dx2);
    const double D3 = interp<0, 0>(g, fp.D[2], i1, dx1, i2, dx2);
    const double B1 = interp<0, 1>(g, fp.B[0], i1, dx1, i2, dx2);
    const double B2 = interp<1, 0>(g, fp.B[1], i1, dx1, i2, dx2);
    const double B3 = interp<1, 1>(g, fp.B[2], i1, dx1, i2, dx2);
    const double al = f.c.alpha;
    const double E[3] = {al * D1 / f.s11, al * f.s22 * D2, al * f.s33 * (f.k13 * D1 + D3)};
    const double B[3] = {al * B1 / f.s11, al * f.s22 * B2, al * f.s33 * (f.k13 * B1 + B3)};
    const double kb = 0.25 * qm * g.dt;
    em_half(f, E, B, kb, u1, u2, u3);
    geodesic_u(g, f, d, u1, u2, u3);
    em_half(f, E, B, kb, u1, u2, u3);
  } else {
    geodesic_u(g, f, d, u1, u2, u3);
  }

  // implicit coordinate update (eq. discretized-geodesic-x); an iterate that
  // repeats exactly is the fixed point of the map, so stopping there gives the
  // same result as running all n_iter iterations (and with iter_tol > 0 the
  // loop also ends once the FP64 change is below the relative tolerance)
  double d1 = 0.0, d2 = 0.0;
  for (int it = 0; it < g.n_iter; ++it) {
    const Coeffs m = coeffs_from(g, rsc_near<FAST>(g, tab, i1, x1 + 0.5 * d1, i2, x2 + 0.5 * d2));
    const double iu0 = m.alpha * rsqrt(1.0 + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 +
                                       m.hu33 * u3 * u3 + 2.0 * m.hu13 * u1 * u3);
    const double n1 = g.dt * ((m.hu11 * u1 + m.hu13 * u3) * iu0 - m.beta1);
    const double n2 = g.dt * (m.hu22 * u2 * iu0);
    const bool fixed = (n1 == d1 && n2 == d2) ||
                       fabs(n1 - d1) + fabs(n2 - d2) <= g.iter_tol * (fabs(n1) + fabs(n2));
    d1 = n1;
    d2 = n2;
    if (fixed) break;
  }
  {
    const Coeffs m = coeffs_from(g, rsc_near<FAST>(g, tab, i1, x1 + 0.5 * d1, i2, x2 + 0.5 * d2));
    const double iu0 = m.alpha * rsqrt(1.0 + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 +
                                       m.hu33 * u3 * u3 + 2.0 * m.hu13 * u1 * u3);
    P.phi[k] += g.dt * (m.hu13 * u1 + m.hu33 * u3) * iu0;
  }
  dx1 += d1;
  renormalize(i1, dx1);
  dx2 += d2;
  renormalize(i2, dx2);
  if (i2 < 0) {
    i2 = 0;
    dx2 = 1.0 - dx2;
    u2 = -u2;
  } else if (i2 >= g.n_th) {
    i2 = g.n_th - 1;
    dx2 = 1.0 - dx2;
    u2 = -u2;
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
}

struct CurrentPlanes {
  double* __restrict__ J[3];
};

__device__ inline void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

// Zigzag charge-conserving deposit (Umeda et al. 2003) in code coordinates
// from the previous to the current position, plus J^3 = q alpha u^3 / gamma at
// the path midpoint with first-order node weights.
//
// A block first accumulates its particles' contributions in a shared-memory
// tile of kTI x kTJ nodes per component (LDS atomics), then adds each touched
// tile node to the global planes once.  Particles sorted by cell make the
// block's footprint small; a block whose footprint exceeds the tile adds
// directly to global memory.
constexpr int kDepBlock = 256;
constexpr int kTI = 8, kTJ = 48;

struct Contrib {
  int ia, ja;         // previous cell: anchor of the 4 x 4 footprint [ia-1, ia+2] x [ja-1, ja+2]
  int di, dj, km, lm; // cell step, J^3 node corner (relative to the anchor)
  double j1[4], j2[4], j3[4];
};

template <bool FAST>
__device__ inline bool make_contrib(const Grid& g, const Tables& tab, const ParticleArrays& P,
                                    int64_t k, Contrib& c) {
  if (k >= P.n) return false;
  const uint8_t t = P.tag[k];
  if (!is_live(t)) return false;
  const double sg = species_sign(t);
  if (sg == 0.0) return false;
  const int ia = P.i1p[k], ja = P.i2p[k];
  const int di = P.i1[k] - ia, dj = P.i2[k] - ja;
  // the zigzag touches at most cells ia-1 .. ia+2: both ends must be in range
  if (!in_grid(g, ia, P.dx1p[k], ja, P.dx2p[k]) ||
      !in_deposit_range(g, P.i1[k], P.dx1[k], P.i2[k], P.dx2[k]) || abs(di) > 1 || abs(dj) > 1)
    return false;
  const double q = sg * g.charge_scale * P.w[k];
  const double qdt = q / g.dt;
  const double xa = P.dx1p[k], ya = P.dx2p[k];
  const double xb = (double)di + P.dx1[k], yb = (double)dj + P.dx2[k];
  const double xr = fmin((double)min(0, di) + 1.0, fmax((double)max(0, di), 0.5 * (xa + xb)));
  const double yr = fmin((double)min(0, dj) + 1.0, fmax((double)max(0, dj), 0.5 * (ya + yb)));
  const double fx1 = qdt * (xr - xa), fy1 = qdt * (yr - ya);
  const double fx2 = qdt * (xb - xr), fy2 = qdt * (yb - yr);
  const double wx1 = 0.5 * (xa + xr), wy1 = 0.5 * (ya + yr);
  const double wx2 = 0.5 * (xr + xb) - di, wy2 = 0.5 * (yr + yb) - dj;
  c.ia = ia;
  c.ja = ja;
  c.di = di;
  c.dj = dj;
  // J^1 at (ia, ja), (ia, ja+1), (ib, jb), (ib, jb+1); J^2 at (ia, ja), (ia+1, ja), (ib, jb), (ib+1, jb)
  c.j1[0] = fx1 * (1.0 - wy1);
  c.j1[1] = fx1 * wy1;
  c.j1[2] = fx2 * (1.0 - wy2);
  c.j1[3] = fx2 * wy2;
  c.j2[0] = fy1 * (1.0 - wx1);
  c.j2[1] = fy1 * wx1;
  c.j2[2] = fy2 * (1.0 - wx2);
  c.j2[3] = fy2 * wx2;
  const double xm = 0.5 * (xa + xb), ym = 0.5 * (ya + yb);
  const Coeffs m = coeffs_from(g, rsc_near<FAST>(g, tab, ia, (double)ia + xm, ja, (double)ja + ym));
  const double u1 = P.u1[k], u2 = P.u2[k], u3 = P.u3[k];
  const double iu0 = m.alpha * rsqrt(1.0 + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 + m.hu33 * u3 * u3 +
                                     2.0 * m.hu13 * u1 * u3);
  const double vphi = (m.hu13 * u1 + m.hu33 * u3) * iu0;
  const double fm = floor(xm), gm = floor(ym);
  const double w1 = xm - fm, w2 = ym - gm;
  const double c3 = q * vphi;
  c.km = (int)fm;
  c.lm = (int)gm;
  // J^3 at (km, lm), (km, lm+1), (km+1, lm), (km+1, lm+1)
  c.j3[0] = c3 * (1.0 - w1) * (1.0 - w2);
  c.j3[1] = c3 * (1.0 - w1) * w2;
  c.j3[2] = c3 * w1 * (1.0 - w2);
  c.j3[3] = c3 * w1 * w2;
  return true;
}

// Adds a contribution through `add(component, i, j, value)` (absolute node indices).
template <class Add>
__device__ inline void scatter(const Contrib& c, Add add) {
  const int ia = c.ia, ja = c.ja, ib = c.ia + c.di, jb = c.ja + c.dj;
  add(0, ia, ja, c.j1[0]);
  add(0, ia, ja + 1, c.j1[1]);
  add(0, ib, jb, c.j1[2]);
  add(0, ib, jb + 1, c.j1[3]);
  add(1, ia, ja, c.j2[0]);
  add(1, ia + 1, ja, c.j2[1]);
  add(1, ib, jb, c.j2[2]);
  add(1, ib + 1, jb, c.j2[3]);
  const int km = ia + c.km, lm = ja + c.lm;
  add(2, km, lm, c.j3[0]);
  add(2, km, lm + 1, c.j3[1]);
  add(2, km + 1, lm, c.j3[2]);
  add(2, km + 1, lm + 1, c.j3[3]);
}

template <bool FAST>
__global__ void __launch_bounds__(kDepBlock) deposit_kernel(Grid g, Tables tab, ParticleArrays P,
                                                            CurrentPlanes cp) {
  __shared__ double tile[3][kTI][kTJ];
  __shared__ int bound[4][kDepBlock / 64];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Contrib c;
  const bool act = make_contrib<FAST>(g, tab, P, k, c);
  // block footprint: union of [ia-1, ia+2] x [ja-1, ja+2]
  int v[4] = {act ? c.ia - 1 : INT_MAX, act ? -(c.ia + 2) : INT_MAX, act ? c.ja - 1 : INT_MAX,
              act ? -(c.ja + 2) : INT_MAX};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    for (int off = 32; off > 0; off >>= 1) v[q] = min(v[q], __shfl_down(v[q], off, 64));
    if (lane == 0) bound[q][wv] = v[q];
  }
  // zero the tile while the bounds settle
  double* flat = &tile[0][0][0];
  for (int e = threadIdx.x; e < 3 * kTI * kTJ; e += kDepBlock) flat[e] = 0.0;
  __syncthreads();
  int b[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    b[q] = bound[q][0];
    for (int w = 1; w < kDepBlock / 64; ++w) b[q] = min(b[q], bound[q][w]);
  }
  const int i0 = b[0], i1 = -b[1], j0 = b[2], j1 = -b[3];
  if (i0 == INT_MAX) return;  // no live charged particle in this block (uniform)
  const bool fits = (i1 - i0 < kTI) && (j1 - j0 < kTJ);
  if (!fits) {
    if (act)
      scatter(c, [&](int comp, int i, int j, double val) { atomic_add(cp.J[comp] + ix(g, i, j), val); });
    return;
  }
  if (act)
    scatter(c, [&](int comp, int i, int j, double val) { atomicAdd(&tile[comp][i - i0][j - j0], val); });
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * kTI * kTJ; e += kDepBlock) {
    const double val = flat[e];
    if (val != 0.0) {
      const int comp = e / (kTI * kTJ), rem = e % (kTI * kTJ);
      atomic_add(cp.J[comp] + ix(g, i0 + rem / kTJ, j0 + rem % kTJ), val);
    }
  }
}

}  // namespace grpic
