// adjoint.hpp -- adjoint of one particle update in a frozen field (the
// differentiation form).
//
// The state of a particle is s = (x1, x2, u1, u2, u3), x = cell + offset; the
// field is F = B0 F1.  One step s' = Phi(s, B0) is Sec. 3.1 steps 2-10 with
// the axis reflection and removal of Sec. 3.3.3.  For each particle the kernel
// rebuilds the step's Jacobian J = d(s')/d(s, B0) (5 x 6) at the stored state
// and returns the vector-Jacobian product
//   gbar(s) = J_s^T gbar(s'),   gbar(B0) += J_B0 . gbar(s').
// The Jacobian propagates six tangent directions through the explicit parts
// of the step (metric and tetrad, gather, the two EM half steps) and takes
// the two implicit-midpoint stages by the implicit-function theorem at their
// converged fixed points:
//   momentum:    Z = u*_{12} + dt f(x, (u* + Z)/2)
//                dZ = (I - dt/2 df/dubar)^-1 (du* + dt df|_{Z fixed})
//   coordinates: d = dt v(x + d/2, u)
//                dd = (I - dt/2 dv/dx)^-1 dt dv|_{d fixed}
// An iteration that did not reach its fixed point within n_iter (no exact
// repeat: next to the axis the contraction can approach 1) is differentiated
// through the iterations the forward pass actually ran instead (tangents
// carried through each of them), so the result is always the derivative of
// the computed map.
// Second derivatives of the metric come from the tangents of the analytic
// first derivatives (frame_from on tangent values).
#pragma once

#include "particles.hpp"
#include "tangent.hpp"

namespace grpic {

constexpr int kAdjDirs = 6;  // x1, x2, u1, u2, u3, B0
using T6 = Tan<kAdjDirs>;
using T2 = Tan<2>;

// r, sin, cos and the map factors of a tangent position (the quasi-spherical
// map of App. A, reflected beyond either axis as in map_theta; theta clamped:
// a clamped angle is constant, the map factors are not)
template <int N>
__device__ inline RSCT<Tan<N>> rsc_tan(const Grid& g, const Tan<N>& x1, const Tan<N>& x2) {
  using TN = Tan<N>;
  RSCT<TN> p;
  const TN e = exp(TN(g.xi_min) + x1 * TN(g.dxi));
  p.r = TN(g.r0) + e;
  p.rd = TN(g.dxi) * e;
  double sg = 1.0, off = 0.0;
  TN xr = x2;
  if (x2.v < 0.0) {
    xr = -x2;
    sg = -1.0;
  } else if (x2.v > (double)g.n_th) {
    xr = TN(2.0 * g.n_th) - x2;
    sg = -1.0;
    off = 2.0 * kPi;
  }
  const TN eta = xr * TN(g.dth), y = eta * TN(1.0 / kPi);
  const double h0 = g.h0;
  TN th = TN(off) + TN(sg) * (eta + TN(2.0 * h0) * eta * (TN(kPi) - TN(2.0) * eta) *
                                        (TN(kPi) - eta) / TN(kPi * kPi));
  p.td = TN(g.dth) * (TN(1.0 + 2.0 * h0) + TN(12.0 * h0) * y * (y - TN(1.0)));
  p.itd2 = rcp(p.td * p.td);
  p.dtd = TN(sg * g.dth * g.dth * 12.0 * h0 / kPi) * (TN(2.0) * y - TN(1.0));
  if (th.v < g.small_angle) th = TN(g.small_angle);
  if (th.v > kPi - g.small_angle) th = TN(kPi - g.small_angle);
  sincos(th, &p.s, &p.c);
  return p;
}

template <int N>
__device__ inline FrameT<double> value_of(const FrameT<Tan<N>>& f) {
  FrameT<double> o;
  o.c = CoeffsT<double>{f.c.alpha.v, f.c.beta1.v, f.c.hu11.v, f.c.hu22.v, f.c.hu33.v, f.c.hu13.v};
  o.s11 = f.s11.v;
  o.s22 = f.s22.v;
  o.s33 = f.s33.v;
  o.k13 = f.k13.v;
  return o;
}

template <int N>
__device__ inline GradT<double> value_of(const GradT<Tan<N>>& d) {
  GradT<double> o;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    o.alpha[q] = d.alpha[q].v;
    o.beta1[q] = d.beta1[q].v;
    o.hu11[q] = d.hu11[q].v;
    o.hu22[q] = d.hu22[q].v;
    o.hu33[q] = d.hu33[q].v;
    o.hu13[q] = d.hu13[q].v;
  }
  return o;
}

template <class R>
__device__ inline GradT<R> lift(const GradT<double>& d) {
  GradT<R> o;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    o.alpha[q] = R(d.alpha[q]);
    o.beta1[q] = R(d.beta1[q]);
    o.hu11[q] = R(d.hu11[q]);
    o.hu22[q] = R(d.hu22[q]);
    o.hu33[q] = R(d.hu33[q]);
    o.hu13[q] = R(d.hu13[q]);
  }
  return o;
}

// Force of the momentum equation (eq. discretized-geodesic-u) at the midpoint
// momentum (b1, b2, u3): f_i = -gamma d_i alpha + b1 d_i beta^1
// - alpha / (2 gamma) d_i h^jk b_j b_k, i = 1, 2.
template <class R>
__device__ inline void geo_force(const CoeffsT<R>& m, const GradT<R>& d, const R& b1, const R& b2,
                                 const R& u3, R fr[2], double mass2) {
  const R Q = R(mass2) + m.hu11 * b1 * b1 + m.hu22 * b2 * b2 + m.hu33 * u3 * u3 +
              R(2.0) * m.hu13 * b1 * u3;
  const R ig = rsqrt(Q);
  const R gb = Q * ig;
  const R h = R(0.5) * m.alpha * ig;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const R q = d.hu11[i] * b1 * b1 + d.hu22[i] * b2 * b2 + d.hu33[i] * u3 * u3 +
                R(2.0) * d.hu13[i] * b1 * u3;
    fr[i] = -(gb * d.alpha[i]) + b1 * d.beta1[i] - h * q;
  }
}

// coordinate velocity (v1, v2) = alpha h^ij u_j / gamma - beta^i
template <class R>
__device__ inline void coord_vel(const CoeffsT<R>& m, const R& u1, const R& u2, const R& u3, R v[2],
                                 double mass2) {
  const R Q = R(mass2) + m.hu11 * u1 * u1 + m.hu22 * u2 * u2 + m.hu33 * u3 * u3 +
              R(2.0) * m.hu13 * u1 * u3;
  const R iu0 = m.alpha * rsqrt(Q);
  v[0] = (m.hu11 * u1 + m.hu13 * u3) * iu0 - m.beta1;
  v[1] = m.hu22 * u2 * iu0;
}

// dz = (I - A)^-1 b for each tangent direction (A 2 x 2)
__device__ inline void solve2(const double A[2][2], T6& z1, T6& z2) {
  const double a = 1.0 - A[0][0], b = -A[0][1], c = -A[1][0], e = 1.0 - A[1][1];
  const double idet = 1.0 / (a * e - b * c);
#pragma unroll
  for (int k = 0; k < kAdjDirs; ++k) {
    const double r1 = z1.d[k], r2 = z2.d[k];
    z1.d[k] = (e * r1 - b * r2) * idet;
    z2.d[k] = (a * r2 - c * r1) * idet;
  }
}

// Bilinear gather with its derivatives in x1, x2 (reading R2); the B0 tangent
// of a field F = B0 F1 is F / B0.
template <int H1, int H2>
__device__ inline T6 interp_tan(const Grid& g, const double* __restrict__ F, int i1, double dx1, int i2,
                                double dx2, double inv_B0) {
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
  const double a0 = f00 + w2 * (f01 - f00), a1 = f10 + w2 * (f11 - f10);
  T6 r(a0 + w1 * (a1 - a0));
  r.d[0] = a1 - a0;
  r.d[1] = (f01 - f00) + w1 * ((f11 - f10) - (f01 - f00));
  r.d[5] = r.v * inv_B0;
  return r;
}

// One particle: gbar_out = J_s^T gbar_in, gB0 += J_B0 . gbar_in.
__device__ inline void adjoint_one(const Grid& g, const GatherPlanesT<double>& fp, double inv_B0,
                                   const ParticleArrays& P, int64_t k, const double gin[5],
                                   double gout[5], double* gB0) {
  const uint8_t t = P.tag[k];
#pragma unroll
  for (int c = 0; c < 5; ++c) gout[c] = gin[c];
  // empty, removed or leaving particles are not moved by the step: identity
  if (!is_live(t) || (t & kLeaving)) return;
  const int i1 = P.i1[k], i2 = P.i2[k];
  const double dx1 = P.dx1[k], dx2 = P.dx2[k];
  if (!in_grid(g, i1, dx1, i2, dx2)) return;
  const T6 x1 = seed<kAdjDirs>((double)i1 + dx1, 0);
  const T6 x2 = seed<kAdjDirs>((double)i2 + dx2, 1);
  T6 u1 = seed<kAdjDirs>(P.u1[k], 2), u2 = seed<kAdjDirs>(P.u2[k], 3), u3 = seed<kAdjDirs>(P.u3[k], 4);

  FrameT<T6> f;
  GradT<T6> d;
  frame_from(g, rsc_tan(g, x1, x2), &f, &d);
  const double qm = species_sign(t);
  const double ms = mass2_of(t);  // m^2 in gamma: 0 for a massless neutral particle
  T6 E[3], B[3];
  if (qm != 0.0) {
    const T6 D1 = interp_tan<1, 0>(g, fp.D[0], i1, dx1, i2, dx2, inv_B0);
    const T6 D2 = interp_tan<0, 1>(g, fp.D[1], i1, dx1, i2, dx2, inv_B0);
    const T6 D3 = interp_tan<0, 0>(g, fp.D[2], i1, dx1, i2, dx2, inv_B0);
    const T6 B1 = interp_tan<0, 1>(g, fp.B[0], i1, dx1, i2, dx2, inv_B0);
    const T6 B2 = interp_tan<1, 0>(g, fp.B[1], i1, dx1, i2, dx2, inv_B0);
    const T6 B3 = interp_tan<1, 1>(g, fp.B[2], i1, dx1, i2, dx2, inv_B0);
    const T6 al = f.c.alpha;
    E[0] = al * D1 / f.s11;
    E[1] = al * f.s22 * D2;
    E[2] = al * f.s33 * (f.k13 * D1 + D3);
    B[0] = al * B1 / f.s11;
    B[1] = al * f.s22 * B2;
    B[2] = al * f.s33 * (f.k13 * B1 + B3);
    em_half(f, E, B, T6(0.25 * qm * g.dt), u1, u2, u3);
  }

  // momentum stage: fixed point in FP64, tangents by the implicit-function theorem
  {
    const FrameT<double> fv = value_of(f);
    const GradT<double> dv = value_of(d);
    const double s1 = u1.v, s2 = u2.v, w3 = u3.v;
    double z1 = s1, z2 = s2;
    bool converged = false;
    for (int it = 0; it < g.n_iter; ++it) {
      double fr[2];
      geo_force(fv.c, dv, 0.5 * (s1 + z1), 0.5 * (s2 + z2), w3, fr, ms);
      const double n1 = s1 + g.dt * fr[0], n2 = s2 + g.dt * fr[1];
      converged = n1 == z1 && n2 == z2;
      z1 = n1;
      z2 = n2;
      if (converged) break;
    }
    if (!converged) {
      // not at the fixed point: tangents through the n_iter iterations run
      T6 t1 = u1, t2 = u2;
      for (int it = 0; it < g.n_iter; ++it) {
        T6 fr[2];
        geo_force(f.c, d, T6(0.5) * (u1 + t1), T6(0.5) * (u2 + t2), u3, fr, ms);
        t1 = u1 + T6(g.dt) * fr[0];
        t2 = u2 + T6(g.dt) * fr[1];
      }
      u1 = t1;
      u2 = t2;
    } else {
      // tangent of the map with Z held fixed
      T6 b1 = T6(0.5) * (u1 + T6(z1)), b2 = T6(0.5) * (u2 + T6(z2));
      T6 fr[2];
      geo_force(f.c, d, b1, b2, u3, fr, ms);
      T6 n1 = u1 + T6(g.dt) * fr[0], n2 = u2 + T6(g.dt) * fr[1];
      // A = dt/2 df/dubar_{12} at the fixed point
      CoeffsT<T2> m2{T2(fv.c.alpha), T2(fv.c.beta1), T2(fv.c.hu11), T2(fv.c.hu22), T2(fv.c.hu33),
                     T2(fv.c.hu13)};
      const GradT<T2> d2 = lift<T2>(dv);
      T2 f2[2];
      geo_force(m2, d2, seed<2>(0.5 * (s1 + z1), 0), seed<2>(0.5 * (s2 + z2), 1), T2(w3), f2, ms);
      const double A[2][2] = {{0.5 * g.dt * f2[0].d[0], 0.5 * g.dt * f2[0].d[1]},
                              {0.5 * g.dt * f2[1].d[0], 0.5 * g.dt * f2[1].d[1]}};
      n1.v = z1;
      n2.v = z2;
      solve2(A, n1, n2);
      u1 = n1;
      u2 = n2;
    }
  }
  if (qm != 0.0) em_half(f, E, B, T6(0.25 * qm * g.dt), u1, u2, u3);

  // coordinate stage
  T6 d1, d2;
  {
    const double a1 = x1.v, a2 = x2.v;
    double e1 = 0.0, e2 = 0.0;
    bool converged = false;
    for (int it = 0; it < g.n_iter; ++it) {
      const CoeffsT<double> m = coeffs_from(g, rsc_direct(g, a1 + 0.5 * e1, a2 + 0.5 * e2));
      double v[2];
      coord_vel(m, u1.v, u2.v, u3.v, v, ms);
      const double n1 = g.dt * v[0], n2 = g.dt * v[1];
      converged = n1 == e1 && n2 == e2;
      e1 = n1;
      e2 = n2;
      if (converged) break;
    }
    if (!converged) {
      // tangents through the n_iter iterations run
      d1 = T6(0.0);
      d2 = T6(0.0);
      for (int it = 0; it < g.n_iter; ++it) {
        T6 v[2];
        coord_vel(coeffs_from(g, rsc_tan(g, x1 + T6(0.5) * d1, x2 + T6(0.5) * d2)), u1, u2, u3, v, ms);
        d1 = T6(g.dt) * v[0];
        d2 = T6(g.dt) * v[1];
      }
    } else {
      const T6 xm1 = x1 + T6(0.5 * e1), xm2 = x2 + T6(0.5 * e2);
      T6 v[2];
      coord_vel(coeffs_from(g, rsc_tan(g, xm1, xm2)), u1, u2, u3, v, ms);
      d1 = T6(g.dt) * v[0];
      d2 = T6(g.dt) * v[1];
      const CoeffsT<T2> m2 =
          coeffs_from(g, rsc_tan(g, seed<2>(a1 + 0.5 * e1, 0), seed<2>(a2 + 0.5 * e2, 1)));
      T2 v2[2];
      coord_vel(m2, T2(u1.v), T2(u2.v), T2(u3.v), v2, ms);
      const double A[2][2] = {{0.5 * g.dt * v2[0].d[0], 0.5 * g.dt * v2[0].d[1]},
                              {0.5 * g.dt * v2[1].d[0], 0.5 * g.dt * v2[1].d[1]}};
      d1.v = e1;
      d2.v = e2;
      solve2(A, d1, d2);
    }
  }
  T6 y1 = x1 + d1, y2 = x2 + d2;
  // axis reflection: x2 -> -x2 below theta = 0, 2 n_th - x2 above theta = pi
  if (floor(y2.v) < 0.0 || floor(y2.v) >= (double)g.n_th) {
    y2 = -y2;
    u2 = -u2;
  }
  const T6* out[5] = {&y1, &y2, &u1, &u2, &u3};
  double gb = 0.0;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 5; ++c) acc += gin[c] * out[c]->d[j];
    gout[j] = acc;
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) gb += gin[c] * out[c]->d[5];
  *gB0 += gb;
}

// gin, gout: 5 x n (SoA rows x1, x2, u1, u2, u3); may alias.  gB0: n, accumulated.
__global__ void __launch_bounds__(64) push_adjoint_kernel(Grid g, GatherPlanesT<double> fp, double inv_B0,
                                                          ParticleArrays P, const double* gin,
                                                          double* gout, double* gB0) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  double a[5], b[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) a[c] = gin[c * P.n + k];
  double acc = gB0[k];
  adjoint_one(g, fp, inv_B0, P, k, a, b, &acc);
#pragma unroll
  for (int c = 0; c < 5; ++c) gout[c * P.n + k] = b[c];
  gB0[k] = acc;
}

}  // namespace grpic
