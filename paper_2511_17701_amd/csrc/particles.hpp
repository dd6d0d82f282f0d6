// particles.hpp -- push and deposit kernels (FP64 form).
//
// One particle per lane; structure-of-arrays loads and stores are contiguous
// across a wavefront.  The push follows Sec. 3.1 steps 1-11 of the paper; the
// deposit Sec. 3.2.
#pragma once

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
    const double gb = sqrt(1.0 + m.hu11 * b1 * b1 + m.hu22 * b2 * b2 + m.hu33 * u33 +
                           2.0 * m.hu13 * b1 * u3);
    const double h = 0.5 * m.alpha / gb;
    double fr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double q = d.hu11[i] * b1 * b1 + d.hu22[i] * b2 * b2 + d.hu33[i] * u33 +
                       2.0 * d.hu13[i] * b1 * u3;
      fr[i] = -gb * d.alpha[i] + b1 * d.beta1[i] - h * q;
    }
    t1 = s1 + g.dt * fr[0];
    t2 = s2 + g.dt * fr[1];
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

__global__ void __launch_bounds__(256) push_kernel(Grid g, GatherPlanes fp, ParticleArrays P) {
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
  frame_at(g, x1, x2, &f, &d);
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

  // implicit coordinate update (eq. discretized-geodesic-x)
  double d1 = 0.0, d2 = 0.0;
  for (int it = 0; it < g.n_iter; ++it) {
    const Coeffs m = coeffs_at(g, x1 + 0.5 * d1, x2 + 0.5 * d2);
    const double iu0 = m.alpha / gamma_of(m, u1, u2, u3);
    d1 = g.dt * ((m.hu11 * u1 + m.hu13 * u3) * iu0 - m.beta1);
    d2 = g.dt * (m.hu22 * u2 * iu0);
  }
  {
    const Coeffs m = coeffs_at(g, x1 + 0.5 * d1, x2 + 0.5 * d2);
    const double iu0 = m.alpha / gamma_of(m, u1, u2, u3);
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
__global__ void __launch_bounds__(256) deposit_kernel(Grid g, ParticleArrays P, CurrentPlanes c) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  const uint8_t t = P.tag[k];
  if (!is_live(t)) return;
  const double sg = species_sign(t);
  if (sg == 0.0) return;
  const double q = sg * g.charge_scale * P.w[k];
  const double qdt = q / g.dt;
  const int ia = P.i1p[k], ja = P.i2p[k];
  const int di = P.i1[k] - ia, dj = P.i2[k] - ja;
  // the zigzag touches at most cells ia-1 .. ia+2: both ends must be in range
  if (!in_grid(g, ia, P.dx1p[k], ja, P.dx2p[k]) ||
      !in_deposit_range(g, P.i1[k], P.dx1[k], P.i2[k], P.dx2[k]) || abs(di) > 1 || abs(dj) > 1)
    return;
  // positions relative to the corner of the previous cell
  const double xa = P.dx1p[k], ya = P.dx2p[k];
  const double xb = (double)di + P.dx1[k], yb = (double)dj + P.dx2[k];
  const double xr = fmin((double)min(0, di) + 1.0, fmax((double)max(0, di), 0.5 * (xa + xb)));
  const double yr = fmin((double)min(0, dj) + 1.0, fmax((double)max(0, dj), 0.5 * (ya + yb)));
  const double fx1 = qdt * (xr - xa), fy1 = qdt * (yr - ya);
  const double fx2 = qdt * (xb - xr), fy2 = qdt * (yb - yr);
  const double wx1 = 0.5 * (xa + xr), wy1 = 0.5 * (ya + yr);
  const double wx2 = 0.5 * (xr + xb) - di, wy2 = 0.5 * (yr + yb) - dj;
  double* J1 = c.J[0];
  double* J2 = c.J[1];
  const int64_t oa = ix(g, ia, ja), ob = ix(g, ia + di, ja + dj);
  atomic_add(J1 + oa, fx1 * (1.0 - wy1));
  atomic_add(J1 + oa + 1, fx1 * wy1);
  atomic_add(J2 + oa, fy1 * (1.0 - wx1));
  atomic_add(J2 + oa + g.ld, fy1 * wx1);
  atomic_add(J1 + ob, fx2 * (1.0 - wy2));
  atomic_add(J1 + ob + 1, fx2 * wy2);
  atomic_add(J2 + ob, fy2 * (1.0 - wx2));
  atomic_add(J2 + ob + g.ld, fy2 * wx2);

  const double xm = 0.5 * (xa + xb), ym = 0.5 * (ya + yb);
  const Coeffs m = coeffs_at(g, (double)ia + xm, (double)ja + ym);
  const double u1 = P.u1[k], u2 = P.u2[k], u3 = P.u3[k];
  const double vphi = (m.hu13 * u1 + m.hu33 * u3) * m.alpha / gamma_of(m, u1, u2, u3);
  const double fm = floor(xm), gm = floor(ym);
  const double w1 = xm - fm, w2 = ym - gm;
  const double c3 = q * vphi;
  double* p3 = c.J[2] + ix(g, ia + (int)fm, ja + (int)gm);
  atomic_add(p3, c3 * (1.0 - w1) * (1.0 - w2));
  atomic_add(p3 + 1, c3 * (1.0 - w1) * w2);
  atomic_add(p3 + g.ld, c3 * w1 * (1.0 - w2));
  atomic_add(p3 + g.ld + 1, c3 * w1 * w2);
}

}  // namespace grpic
