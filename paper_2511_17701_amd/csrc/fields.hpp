// fields.hpp -- field-solver kernels (Sec. 3.3, 3.4).
//
// Kernels are templated on the storage type T of the planes (double, or float
// in the single-precision form); the metric weights and the update arithmetic
// are FP64 and each result is rounded once on store.  The solver is bound by
// plane traffic, so the FP64 arithmetic costs nothing.
//
// Threads run along theta (the contiguous index of a plane), blocks along r.
// Geometry at staggered grid points is assembled from 1-D tables of r at
// integer / half-integer x1 and of sin, cos at integer / half-integer x2.
#pragma once

#include "geometry.hpp"

namespace grpic {

__device__ inline Cell cell_tab(const Grid& g, const Tables& t, int i, int o1, int j, int o2) {
  const double r = t.r[o1][i + g.ng];
  const double s = t.s[o2][j + g.ng], c = t.c[o2][j + g.ng];
  const double a2 = g.a * g.a, r2 = r * r, tMr = 2.0 * g.M * r;
  const double Sig = r2 + a2 * c * c;
  const double S2 = Sig + tMr;
  const double ra = r2 + a2;
  const double A = ra * ra - a2 * (ra - tMr) * s * s;
  const double R = g.dxi * r;
  const double opz = S2 / Sig;
  Cell e;
  e.alpha = sqrt(Sig / S2);
  e.beta1 = tMr / (S2 * R);
  e.hl11 = opz * R * R;
  e.hl22 = Sig * g.dth * g.dth;
  e.hl33 = A * s * s / Sig;
  e.hl13 = -g.a * opz * s * s * R;
  e.sqrt_ht = R * g.dth * Sig / e.alpha;
  e.sqrt_h = e.sqrt_ht * s;
  return e;
}

template <class T>
struct TriT {
  T* __restrict__ p[3];
};
template <class T>
struct CTriT {
  const T* __restrict__ p[3];
};
using Tri = TriT<double>;
using CTri = CTriT<double>;

// X[o] += inc.  In the single-precision form the evolved fields D and B carry
// a compensation plane L (null otherwise): X + L holds the running sum to about
// 48 bits and X, what every reader sees, is its rounding to float, so rounding
// errors of the time integration do not accumulate step after step.
template <class T>
__device__ inline void add_to(T* __restrict__ X, T* __restrict__ L, int64_t o, double inc) {
  if (sizeof(T) == 4 && L) {
    const double v = ((double)X[o] + (double)L[o]) + inc;
    const T h = (T)v;
    X[o] = h;
    L[o] = (T)(v - (double)h);
  } else {
    X[o] = (T)((double)X[o] + inc);
  }
}

// ---------------------------------------------------------------- aux E, H
// eq. discretized-auxE/-auxH with the volume-weighted radial averages of
// Sec. 3.3.1 (weights sqrt(h)/sin(theta)); for i in [-1, n_r], j in [0, n_th].

template <class T>
__global__ void aux_e_kernel(Grid g, Tables t, CTriT<T> Bs, CTriT<T> Ds, TriT<T> E) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y - 1;
  if (j > g.n_th || i > g.n_r) return;
  const int64_t o = ix(g, i, j);
  {  // E_1 (i+1/2, j)
    const Cell c = cell_tab(g, t, i, 1, j, 0);
    const Cell m0 = cell_tab(g, t, i, 0, j, 0), m1 = cell_tab(g, t, i + 1, 0, j, 0);
    const double av = (m0.sqrt_ht * m0.hl13 * Ds.p[2][o] + m1.sqrt_ht * m1.hl13 * Ds.p[2][o + g.ld]) /
                      (2.0 * c.sqrt_ht);
    E.p[0][o] = c.alpha * (c.hl11 * Ds.p[0][o] + av);
  }
  {  // E_3 (i, j)
    const Cell c = cell_tab(g, t, i, 0, j, 0);
    const Cell m0 = cell_tab(g, t, i - 1, 1, j, 0), m1 = cell_tab(g, t, i, 1, j, 0);
    const double w0 = m0.sqrt_ht, w1 = m1.sqrt_ht, iw = 1.0 / (2.0 * c.sqrt_ht);
    const double a1 = (w0 * m0.hl13 * Ds.p[0][o - g.ld] + w1 * m1.hl13 * Ds.p[0][o]) * iw;
    const double a2 = (w0 * m0.sqrt_h * m0.beta1 * Bs.p[1][o - g.ld] +
                       w1 * m1.sqrt_h * m1.beta1 * Bs.p[1][o]) * iw;
    E.p[2][o] = c.alpha * (c.hl33 * Ds.p[2][o] + a1) + a2;
  }
  if (j < g.n_th) {  // E_2 (i, j+1/2)
    const Cell c = cell_tab(g, t, i, 0, j, 1);
    const Cell m0 = cell_tab(g, t, i - 1, 1, j, 1), m1 = cell_tab(g, t, i, 1, j, 1);
    const double a3 = (m0.sqrt_ht * m0.sqrt_h * m0.beta1 * Bs.p[2][o - g.ld] +
                       m1.sqrt_ht * m1.sqrt_h * m1.beta1 * Bs.p[2][o]) / (2.0 * c.sqrt_ht);
    E.p[1][o] = c.alpha * c.hl22 * Ds.p[1][o] - a3;
  }
}

template <class T>
__global__ void aux_h_kernel(Grid g, Tables t, CTriT<T> Bs, CTriT<T> Ds, TriT<T> H) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y - 1;
  if (j > g.n_th || i > g.n_r) return;
  const int64_t o = ix(g, i, j);
  {  // H_2 (i+1/2, j)
    const Cell c = cell_tab(g, t, i, 1, j, 0);
    const Cell m0 = cell_tab(g, t, i, 0, j, 0), m1 = cell_tab(g, t, i + 1, 0, j, 0);
    const double a1 = (m0.sqrt_ht * m0.sqrt_h * m0.beta1 * Ds.p[2][o] +
                       m1.sqrt_ht * m1.sqrt_h * m1.beta1 * Ds.p[2][o + g.ld]) / (2.0 * c.sqrt_ht);
    H.p[1][o] = c.alpha * c.hl22 * Bs.p[1][o] + a1;
  }
  if (j < g.n_th) {
    {  // H_1 (i, j+1/2)
      const Cell c = cell_tab(g, t, i, 0, j, 1);
      const Cell m0 = cell_tab(g, t, i - 1, 1, j, 1), m1 = cell_tab(g, t, i, 1, j, 1);
      const double a2 = (m0.sqrt_ht * m0.hl13 * Bs.p[2][o - g.ld] + m1.sqrt_ht * m1.hl13 * Bs.p[2][o]) /
                        (2.0 * c.sqrt_ht);
      H.p[0][o] = c.alpha * (c.hl11 * Bs.p[0][o] + a2);
    }
    {  // H_3 (i+1/2, j+1/2)
      const Cell c = cell_tab(g, t, i, 1, j, 1);
      const Cell m0 = cell_tab(g, t, i, 0, j, 1), m1 = cell_tab(g, t, i + 1, 0, j, 1);
      const double iw = 1.0 / (2.0 * c.sqrt_ht);
      const double a3 = (m0.sqrt_ht * m0.hl13 * Bs.p[0][o] + m1.sqrt_ht * m1.hl13 * Bs.p[0][o + g.ld]) * iw;
      const double a4 = (m0.sqrt_ht * m0.sqrt_h * m0.beta1 * Ds.p[1][o] +
                         m1.sqrt_ht * m1.sqrt_h * m1.beta1 * Ds.p[1][o + g.ld]) * iw;
      H.p[2][o] = c.alpha * (c.hl33 * Bs.p[2][o] + a3) - a4;
    }
  }
}

// ---------------------------------------------------------------- Faraday
// eq. discretized-faraday on the evolved ranges (thread (i, j), i in [0, n_r],
// j in [0, n_th]).
template <class T>
__global__ void faraday_kernel(Grid g, Tables t, TriT<T> X, TriT<T> L, CTriT<T> E) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (j > g.n_th || i > g.n_r) return;
  const int64_t o = ix(g, i, j);
  if (j < g.n_th) {
    const Cell c = cell_tab(g, t, i, 0, j, 1);
    add_to(X.p[0], L.p[0], o, -(g.dt * (E.p[2][o + 1] - E.p[2][o]) / c.sqrt_h));
  }
  if (i < g.n_r && j >= 1 && j < g.n_th) {
    const Cell c = cell_tab(g, t, i, 1, j, 0);
    add_to(X.p[1], L.p[1], o, g.dt * (E.p[2][o + g.ld] - E.p[2][o]) / c.sqrt_h);
  }
  if (i < g.n_r && j < g.n_th) {
    const Cell c = cell_tab(g, t, i, 1, j, 1);
    const double curl = (E.p[1][o + g.ld] - E.p[1][o]) - (E.p[0][o + 1] - E.p[0][o]);
    add_to(X.p[2], L.p[2], o, -(g.dt * curl / c.sqrt_h));
  }
}

// ---------------------------------------------------------------- Ampere
// eq. discretized-ampere with J = wa Ja + wb Jb; D^1 on the axis rows from the
// polar-cap integral form (Sec. 3.3.2): cap area A_{i+1/2}; the theta = pi cap
// has the opposite orientation, and the one-sided axis-row current enters
// with 4 pi.
template <class T>
__global__ void ampere_kernel(Grid g, Tables t, TriT<T> X, TriT<T> L, CTriT<T> H, CTriT<T> Ja, CTriT<T> Jb, double wa,
                              double wb, double polar_k) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (j > g.n_th || i > g.n_r) return;
  const int64_t o = ix(g, i, j);
  const double fpi = 4.0 * kPi;
  if (i < g.n_r) {
    const double J1 = wa * Ja.p[0][o] + wb * Jb.p[0][o];
    if (j >= 1 && j < g.n_th) {
      const Cell c = cell_tab(g, t, i, 1, j, 0);
      add_to(X.p[0], L.p[0], o, g.dt * ((H.p[2][o] - H.p[2][o - 1]) - fpi * J1) / c.sqrt_h);
    } else {
      const double r = t.r[1][i + g.ng];
      const double ra = r * r + g.a * g.a;
      const double Ap = g.dxi * r * ra * sqrt(1.0 + 2.0 * g.M * r / ra) * polar_k;
      const double h3 = (j == 0) ? H.p[2][o] : -H.p[2][o - 1];
      add_to(X.p[0], L.p[0], o, g.dt * (h3 - fpi * J1) / Ap);
    }
  }
  if (j < g.n_th) {
    const Cell c = cell_tab(g, t, i, 0, j, 1);
    const double J2 = wa * Ja.p[1][o] + wb * Jb.p[1][o];
    add_to(X.p[1], L.p[1], o, g.dt * (-(H.p[2][o] - H.p[2][o - g.ld]) - fpi * J2) / c.sqrt_h);
  }
  if (j >= 1 && j < g.n_th) {
    const Cell c = cell_tab(g, t, i, 0, j, 0);
    const double J3 = wa * Ja.p[2][o] + wb * Jb.p[2][o];
    const double curl = (H.p[1][o] - H.p[1][o - g.ld]) - (H.p[0][o] - H.p[0][o - 1]);
    add_to(X.p[2], L.p[2], o, g.dt * (curl - fpi * J3) / c.sqrt_h);
  }
}

// ---------------------------------------------------------------- boundaries
// Constant layer inside the horizon (i in [-ng, n_f] takes row n_f + 1) and the
// absorbing layer (F <- F - lambda (F - F_init), lambda a cubic ramp over the
// last n_absorb cells); whole plane incl. ghosts.  half1[c] = staggering of
// component c in x1.
template <class T>
__global__ void bc_radial_kernel(Grid g, TriT<T> X, TriT<T> L, CTriT<T> X0, int3 half1) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x - g.ng;
  const int i = blockIdx.y * blockDim.y + threadIdx.y - g.ng;
  if (j >= g.n_th + g.ng || i >= g.n_r + g.ng) return;
  const int64_t o = ix(g, i, j);
  const int hs[3] = {half1.x, half1.y, half1.z};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (i <= g.n_filter) {
      X.p[c][o] = X.p[c][ix(g, g.n_filter + 1, j)];
      if (sizeof(T) == 4 && L.p[c]) L.p[c][o] = L.p[c][ix(g, g.n_filter + 1, j)];
    } else if (g.n_absorb > 0) {
      const double x = (double)i + 0.5 * hs[c];
      const double x0 = (double)(g.n_r - g.n_absorb);
      if (x > x0) {
        const double s = fmin((x - x0) / g.n_absorb, 1.0);
        const double lam = s * s * s;
        if (sizeof(T) == 4 && L.p[c]) {
          const double v = (double)X.p[c][o] + (double)L.p[c][o];
          const double w = v - lam * (v - X0.p[c][o]);
          const T h = (T)w;
          X.p[c][o] = h;
          L.p[c][o] = (T)(w - (double)h);
        } else {
          X.p[c][o] = X.p[c][o] - lam * (X.p[c][o] - X0.p[c][o]);
        }
      }
    }
  }
}

// Axis reflection (Sec. 3.3.3): r-components even, theta and phi components
// odd; with zero_axis, the theta component of B (B^2) or the phi component of
// D (D^3) vanishes on the axis rows.  half2[c] = staggering in x2.
template <class T>
__global__ void bc_axis_kernel(Grid g, TriT<T> X, TriT<T> L, int3 half2, int zero_comp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x - g.ng;
  if (i >= g.n_r + g.ng) return;
  const int hs[3] = {half2.x, half2.y, half2.z};
  const double par[3] = {1.0, -1.0, -1.0};
  const int n = g.n_th;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T* C = X.p[c];
    if (!hs[c]) {
      if (c == zero_comp) {
        C[ix(g, i, 0)] = 0.0;
        C[ix(g, i, n)] = 0.0;
        if (sizeof(T) == 4 && L.p[c]) {
          L.p[c][ix(g, i, 0)] = 0.0;
          L.p[c][ix(g, i, n)] = 0.0;
        }
      }
      // node rows run 0..n: ng ghost rows below the axis, ng - 1 above
      for (int k = 1; k <= g.ng; ++k) C[ix(g, i, -k)] = par[c] * C[ix(g, i, k)];
      for (int k = 1; k < g.ng; ++k) C[ix(g, i, n + k)] = par[c] * C[ix(g, i, n - k)];
    } else {
      for (int k = 1; k <= g.ng; ++k) {
        C[ix(g, i, -k)] = par[c] * C[ix(g, i, k - 1)];
        C[ix(g, i, n - 1 + k)] = par[c] * C[ix(g, i, n - k)];
      }
    }
  }
}

// ---------------------------------------------------------------- misc
// elementwise over ncomp planes (whole planes incl. ghosts)
template <class T>
__global__ void average_kernel(int64_t n, TriT<T> A, CTriT<T> B) {  // A <- (A + B) / 2
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) A.p[c][k] = 0.5 * (A.p[c][k] + B.p[c][k]);
}

template <class T>
__global__ void copy_kernel(int64_t n, TriT<T> A, CTriT<T> B) {  // A <- B
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) A.p[c][k] = B.p[c][k];
}

template <class T>
__global__ void rotate_currents_kernel(int64_t n, TriT<T> J0, TriT<T> J) {  // J0 <- J, J <- 0
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    J0.p[c][k] = J.p[c][k];
    J.p[c][k] = 0.0;
  }
}

template <class T>
__global__ void fill_kernel(int64_t n, T* __restrict__ p, double v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// One binomial pass (1,2,1)/4 x (1,2,1)/4 from S into X for i in
// [1 - ng, n_r + ng - 2], j in [0, n_th - half2[c]].
template <class T>
__global__ void filter_kernel(Grid g, TriT<T> X, CTriT<T> S, int3 half2, int ncomp) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y + 1 - g.ng;
  if (j > g.n_th || i > g.n_r + g.ng - 2) return;
  const int hs[3] = {half2.x, half2.y, half2.z};
  const int64_t o = ix(g, i, j);
  for (int c = 0; c < ncomp; ++c) {
    if (j > g.n_th - hs[c]) continue;
    const T* s = S.p[c];
    const double r0 = s[o - g.ld - 1] + 2.0 * s[o - g.ld] + s[o - g.ld + 1];
    const double r1 = s[o - 1] + 2.0 * s[o] + s[o + 1];
    const double r2 = s[o + g.ld - 1] + 2.0 * s[o + g.ld] + s[o + g.ld + 1];
    X.p[c][o] = 0.0625 * (r0 + 2.0 * r1 + r2);
  }
}

}  // namespace grpic
