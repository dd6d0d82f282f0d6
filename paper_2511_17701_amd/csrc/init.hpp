// init.hpp -- initial data on the device: Wald vacuum field (Sec. 4.1.2) and
// particle loading (Philox4x32-10, Maxwell-Juttner by Sobol's method).
#pragma once

#include "fields.hpp"
#include "particles.hpp"

namespace grpic {

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32
// multiplies (0xD2511F53, 0xCD9E8D57) with a Weyl key schedule (0x9E3779B9,
// 0xBB67AE85).
__host__ __device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// counter (index, sub, stream, attempt), key = seed; sub = 0 for the initial
// loading, 1 + call for the pair-injection call `call`
__device__ inline void draw4(uint64_t seed, uint32_t idx, uint32_t stream, uint32_t k,
                             uint32_t out[4], uint32_t sub = 0u) {
  out[0] = idx;
  out[1] = sub;
  out[2] = stream;
  out[3] = k;
  philox(out, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ inline double u_open0(uint32_t w) { return ((double)w + 1.0) * 0x1p-32; }  // (0, 1]
__device__ inline double u_mid(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }    // (0, 1)
__device__ inline double u_low(uint32_t w) { return (double)w * 0x1p-32; }            // [0, 1)

// Isotropic Maxwell-Juttner spatial 4-velocity at temperature T: Sobol's
// rejection method (as given by Zenitani 2015): u = -T ln(X1 X2 X3),
// eta = -T ln(X1 X2 X3 X4), accept when eta^2 - u^2 > 1; direction from two
// further uniforms.
__device__ inline void maxwell_juttner(uint64_t seed, uint32_t q, double T, double uh[3],
                                       uint32_t sub = 0u) {
  double u = 0.0;
  for (uint32_t k = 0; k < 4096u; ++k) {
    uint32_t w[4];
    draw4(seed, q, 1u, k, w, sub);
    const double x123 = u_open0(w[0]) * u_open0(w[1]) * u_open0(w[2]);
    u = -T * log(x123);
    const double eta = -T * log(x123 * u_open0(w[3]));
    if (eta * eta - u * u > 1.0) break;
  }
  uint32_t w[4];
  draw4(seed, q, 2u, 0u, w, sub);
  const double x5 = u_mid(w[0]), x6 = u_mid(w[1]);
  const double st = 2.0 * u * sqrt(x5 * (1.0 - x5));
  double sn, cs;
  sincos(2.0 * kPi * x6, &sn, &cs);
  uh[0] = u * (2.0 * x5 - 1.0);
  uh[1] = st * cs;
  uh[2] = st * sn;
}

struct Tetrad {
  double s11, s22, s33, k13;
};

// tetrad factors at (x1, x2), theta clamped (App. A)
__device__ inline Tetrad tetrad_at(const Grid& g, double x1, double x2) {
  double r, R, th, T, dT;
  map_r(g, x1, &r, &R);
  map_theta(g, x2, &th, &T, &dT);
  double s, c;
  sincos(clamp_theta(g, th), &s, &c);
  const double a2 = g.a * g.a, r2 = r * r, tMr = 2.0 * g.M * r;
  const double Sig = r2 + a2 * c * c, S2 = Sig + tMr, ra = r2 + a2;
  const double A = ra * ra - a2 * (ra - tMr) * s * s;
  Tetrad e;
  e.s11 = sqrt(A / (Sig * S2)) / R;
  e.s22 = sqrt(Sig) * T;
  e.s33 = sqrt(A / Sig) * s;
  e.k13 = -g.a * R * S2 / A;
  return e;
}

__device__ inline void hat_to_cov(const Tetrad& e, const double uh[3], double& u1, double& u2,
                                  double& u3) {
  u1 = uh[0] / e.s11 + e.k13 * e.s33 * uh[2];
  u2 = e.s22 * uh[1];
  u3 = e.s33 * uh[2];
}

// x2 of a polar angle: theta / dth on the uniform-theta grid; bisection of
// the increasing map of App. A otherwise
__device__ inline double x2_of_theta(const Grid& g, double th) {
  if (g.h0 == 0.0) return th / g.dth;
  double lo = 0.0, hi = (double)g.n_th;
  for (int it = 0; it < 100; ++it) {
    const double mid = 0.5 * (lo + hi);
    double t, td, dtd;
    map_theta(g, mid, &t, &td, &dtd);
    if (t < th) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

template <class T>
__device__ inline void store_particle(ParticleArraysT<T>& P, int64_t q, int i1, int i2, double dx1,
                                      double dx2, double u1, double u2, double u3, uint8_t tag,
                                      double w = 1.0) {
  P.i1[q] = i1;
  P.i2[q] = i2;
  P.dx1[q] = dx1;
  P.dx2[q] = dx2;
  P.i1p[q] = i1;
  P.i2p[q] = i2;
  P.dx1p[q] = dx1;
  P.dx2p[q] = dx2;
  P.u1[q] = u1;
  P.u2[q] = u2;
  P.u3[q] = u3;
  P.w[q] = w;
  P.phi[q] = 0.0;
  P.tag[q] = tag;
}

// One thread per pair k: slots 2k (e+) and 2k+1 (e-) at one position.
template <class T>
__global__ void load_pairs_kernel(Grid g, ParticleArraysT<T> P, int64_t n_pairs, int ppc, double temp,
                                  uint64_t seed) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pairs) return;
  uint32_t w[4];
  draw4(seed, (uint32_t)k, 0u, 0u, w);
  const int64_t ncell = (int64_t)g.n_r * g.n_th;
  const int64_t cell = ppc > 0 ? k / (ppc / 2)
                               : (int64_t)((((uint64_t)w[2] << 32) | w[3]) % (uint64_t)ncell);
  const int i1 = (int)(cell / g.n_th), i2 = (int)(cell % g.n_th);
  const double dx1 = u_low(w[0]), dx2 = u_low(w[1]);
  const Tetrad e = tetrad_at(g, (double)i1 + dx1, (double)i2 + dx2);
  for (int s = 0; s < 2; ++s) {
    const int64_t q = 2 * k + s;
    double uh[3], u1, u2, u3;
    maxwell_juttner(seed, (uint32_t)q, temp, uh);
    hat_to_cov(e, uh, u1, u2, u3);
    store_particle(P, q, i1, i2, dx1, dx2, u1, u2, u3, (uint8_t)(s == 0 ? 1 : 2));
  }
}

// Neutral bound test particles (tag 3): r in U[6, 15], theta in U[pi/3, 2pi/3],
// tetrad velocity (0.05 U[-1,1], 0.05 U[-1,1], (0.9 + 0.2 U) sqrt(M/(r - 3M))),
// redrawn until E = alpha gamma - beta^1 u_1 < 1.
template <class T>
__global__ void load_geodesics_kernel(Grid g, ParticleArraysT<T> P, int64_t first, int64_t n_geo,
                                      uint64_t seed) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_geo) return;
  int i1 = 0, i2 = 0;
  double dx1 = 0.0, dx2 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
  for (uint32_t a = 0; a < 64u; ++a) {
    uint32_t w[4], v[4];
    draw4(seed, (uint32_t)k, 3u, a, w);
    draw4(seed, (uint32_t)k, 4u, a, v);
    const double r = 6.0 + 9.0 * u_low(w[0]);
    const double th = kPi / 3.0 + (kPi / 3.0) * u_low(w[1]);
    const double x1 = (log(r - g.r0) - g.xi_min) / g.dxi, x2 = x2_of_theta(g, th);
    const double f1 = floor(x1), f2 = floor(x2);
    i1 = (int)f1;
    dx1 = x1 - f1;
    i2 = (int)f2;
    dx2 = x2 - f2;
    const double y1 = (double)i1 + dx1, y2 = (double)i2 + dx2;
    const Tetrad e = tetrad_at(g, y1, y2);
    const double rr = g.r0 + exp(g.xi_min + y1 * g.dxi);
    const double uk = sqrt(g.M / (rr - 3.0 * g.M));
    const double uh[3] = {0.05 * (2.0 * u_low(w[3]) - 1.0), 0.05 * (2.0 * u_low(v[0]) - 1.0),
                          (0.9 + 0.2 * u_low(w[2])) * uk};
    hat_to_cov(e, uh, u1, u2, u3);
    const Coeffs m = coeffs_at(g, y1, y2);
    const double E = m.alpha * gamma_of(m, u1, u2, u3) - m.beta1 * u1;
    if (E < 1.0) break;
  }
  store_particle(P, first + k, i1, i2, dx1, dx2, u1, u2, u3, 3);
}

// ------------------------------------------------------------------ Wald
// A_mu = (B0/2)(g_mu3 + 2 a g_mu0) in Kerr-Schild components (eq. Wald):
//   A_0 = (B0 a/2)(z (1 + cos^2) - 2), A_r = (B0 a/2)(2 z - (1 + z) sin^2),
//   A_3 = (B0/2) sin^2 (A/Sigma - 2 a^2 z),  z = 2 M r / Sigma.
struct WaldPot {
  double A0, Ar, A3;        // values
  double A0_r, A0_t;        // d A_0 / dr, d A_0 / dtheta
  double A3_r, A3_t, Ar_t;  // d A_3 / dr, d A_3 / dtheta, d A_r / dtheta
};

__device__ inline WaldPot wald_pot(const Grid& g, double r, double s, double c, double B0) {
  const double a = g.a, M = g.M, a2 = a * a, r2 = r * r;
  const double Sig = r2 + a2 * c * c, iSig = 1.0 / Sig;
  const double ra = r2 + a2, Del = ra - 2.0 * M * r;
  const double A = ra * ra - a2 * Del * s * s;
  const double z = 2.0 * M * r * iSig;
  const double Sig_t = -2.0 * a2 * s * c;
  const double z_r = 2.0 * M * (Sig - 2.0 * r2) * iSig * iSig;
  const double z_t = -z * Sig_t * iSig;
  const double A_r = 4.0 * r * ra - a2 * s * s * (2.0 * r - 2.0 * M);
  const double A_t = -2.0 * a2 * Del * s * c;
  const double hb = 0.5 * B0, hba = 0.5 * B0 * a;
  WaldPot p;
  p.A0 = hba * (z * (1.0 + c * c) - 2.0);
  p.A0_r = hba * z_r * (1.0 + c * c);
  p.A0_t = hba * (z_t * (1.0 + c * c) - 2.0 * z * s * c);
  p.Ar = hba * (2.0 * z - (1.0 + z) * s * s);
  p.Ar_t = hba * (z_t * (2.0 - s * s) - 2.0 * (1.0 + z) * s * c);
  const double Q = A * iSig - 2.0 * a2 * z;
  const double Q_r = (A_r - A * 2.0 * r * iSig) * iSig - 2.0 * a2 * z_r;
  const double Q_t = (A_t - A * Sig_t * iSig) * iSig - 2.0 * a2 * z_t;
  p.A3 = hb * s * s * Q;
  p.A3_r = hb * s * s * Q_r;
  p.A3_t = hb * (2.0 * s * c * Q + s * s * Q_t);
  return p;
}

struct PotCode {
  double A1, A3;  // code components: A_1 = (dr/dx1) A_r, A_3
};

__device__ inline PotCode wald_code(const Grid& g, double x1, double x2, double B0) {
  double r, R, th, T, dT;
  map_r(g, x1, &r, &R);
  map_theta(g, x2, &th, &T, &dT);
  double s, c;
  sincos(th, &s, &c);
  const WaldPot p = wald_pot(g, r, s, c, B0);
  return PotCode{p.Ar * R, p.A3};
}

// analytic D^i (component comp) at (x1, x2): E_i = d_i A_0 and
// sqrt(h) B^k from the curl of A, D^j = h^ji (E_i - e_ikl beta^k B^l) / alpha
__device__ inline double wald_D(const Grid& g, double x1, double x2, double B0, int comp) {
  double r, R, th, T, dT;
  map_r(g, x1, &r, &R);
  map_theta(g, x2, &th, &T, &dT);
  double s, c;
  sincos(th, &s, &c);
  const WaldPot p = wald_pot(g, r, s, c, B0);
  const double a2 = g.a * g.a, r2 = r * r, tMr = 2.0 * g.M * r;
  const double Sig = r2 + a2 * c * c, S2 = Sig + tMr, ra = r2 + a2;
  const double A = ra * ra - a2 * (ra - tMr) * s * s;
  const double alpha = sqrt(Sig / S2);
  const double beta1 = tMr / (S2 * R);
  // code derivatives: d/dx1 = R d/dr, d/dx2 = T d/dtheta
  const double E1 = R * p.A0_r, E2 = T * p.A0_t;
  const double shB2 = -R * p.A3_r;          // sqrt(h) B^2
  const double shB3 = -T * R * p.Ar_t;      // sqrt(h) B^3
  const double X1 = E1;
  const double X2 = E2 + beta1 * shB3;
  const double X3 = -beta1 * shB2;
  if (comp == 0) return (A / (Sig * S2) / (R * R) * X1 + g.a / (Sig * R) * X3) / alpha;
  if (comp == 1) return 1.0 / (T * T) / Sig * X2 / alpha;
  return (g.a / (Sig * R) * X1 + X3 / (Sig * s * s)) / alpha;
}

__device__ inline double wald_B(const Grid& g, double x1, double x2, double B0, int comp) {
  double r, R, th, T, dT;
  map_r(g, x1, &r, &R);
  map_theta(g, x2, &th, &T, &dT);
  double s, c;
  sincos(th, &s, &c);
  const WaldPot p = wald_pot(g, r, s, c, B0);
  const double a2 = g.a * g.a, r2 = r * r;
  const double Sig = r2 + a2 * c * c, S2 = Sig + 2.0 * g.M * r;
  const double sqrt_h = R * T * Sig * s / sqrt(Sig / S2);
  if (comp == 0) return T * p.A3_t / sqrt_h;
  if (comp == 1) return -R * p.A3_r / sqrt_h;
  return -T * R * p.Ar_t / sqrt_h;
}

// Whole planes incl. ghosts: D pointwise, B by the discrete Stokes curl of
// A_3 (nodes) and A_1 (r-edges); the last row/column (no neighbour) takes the
// analytic B.
template <class T>
__global__ void wald_kernel(Grid g, Tables t, TriT<T> D, TriT<T> B, double B0) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x - g.ng;
  const int i = blockIdx.y * blockDim.y + threadIdx.y - g.ng;
  if (j >= g.n_th + g.ng || i >= g.n_r + g.ng) return;
  const int64_t o = ix(g, i, j);
  D.p[0][o] = wald_D(g, i + 0.5, j, B0, 0);
  D.p[1][o] = wald_D(g, i, j + 0.5, B0, 1);
  D.p[2][o] = wald_D(g, i, j, B0, 2);
  const bool last_i = i == g.n_r + g.ng - 1, last_j = j == g.n_th + g.ng - 1;
  if (!last_j) {
    const Cell c = cell_tab(g, t, i, 0, j, 1);
    B.p[0][o] = (wald_code(g, i, j + 1, B0).A3 - wald_code(g, i, j, B0).A3) / c.sqrt_h;
  } else {
    B.p[0][o] = wald_B(g, i, j + 0.5, B0, 0);
  }
  if (!last_i) {
    const Cell c = cell_tab(g, t, i, 1, j, 0);
    B.p[1][o] = -(wald_code(g, i + 1, j, B0).A3 - wald_code(g, i, j, B0).A3) / c.sqrt_h;
  } else {
    B.p[1][o] = wald_B(g, i + 0.5, j, B0, 1);
  }
  if (!last_j) {
    const Cell c = cell_tab(g, t, i, 1, j, 1);
    B.p[2][o] = -(wald_code(g, i + 0.5, j + 1, B0).A1 - wald_code(g, i + 0.5, j, B0).A1) / c.sqrt_h;
  } else {
    B.p[2][o] = wald_B(g, i + 0.5, j + 0.5, B0, 2);
  }
}

// Monopole initial data of the BZ test: A_phi = -B0 cos(theta), so B^1 at
// (i, j+1/2) is the difference of A_3 between the nodes j and j+1 over sqrt(h)
// (eq. EB-set) and every other component is zero (the caller zeroes the
// planes).  The last column (no node j+1) takes the analytic
// B^1 = T B0 sin(theta) / sqrt(h), T = dtheta/dx2; the axis pass overwrites it.
template <class T>
__global__ void monopole_kernel(Grid g, Tables t, T* __restrict__ B1, double B0) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x - g.ng;
  const int i = blockIdx.y * blockDim.y + threadIdx.y - g.ng;
  if (j >= g.n_th + g.ng || i >= g.n_r + g.ng) return;
  const double sqrt_h = cell_tab(g, t, i, 0, j, 1).sqrt_h;
  double v;
  if (j < g.n_th + g.ng - 1) {
    const double a3 = -B0 * t.c[0][j + g.ng], b3 = -B0 * t.c[0][j + 1 + g.ng];
    v = (b3 - a3) / sqrt_h;
  } else {
    v = t.td[1][j + g.ng] * B0 * t.s[1][j + g.ng] / sqrt_h;
  }
  B1[ix(g, i, j)] = (T)v;
}

}  // namespace grpic
