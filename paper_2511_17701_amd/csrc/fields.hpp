// fields.hpp -- field-solver kernels (Sec. 3.3, 3.4).
//
// Kernels are templated on the storage type T of the planes (double, or float
// in the single-precision form); the metric weights and the update arithmetic
// are FP64 and each result is rounded once on store.
//
// Threads run along theta (the contiguous index of a plane), blocks along r.
// Geometry at staggered grid points is assembled from 1-D tables of r and
// 1/(R deta) at integer / half-integer x1 and of sin, cos, 1/sin (and, when
// h0 != 0, T = dtheta/dx2 and deta/T) at integer / half-integer x2, with one
// reciprocal square root per point; R = dr/dx1 = dxi (r - r0).
#pragma once

#include "geometry.hpp"

namespace grpic {

__device__ inline Cell cell_tab(const Grid& g, const Tables& t, int i, int o1, int j, int o2) {
  const double r = t.r[o1][i + g.ng], R = g.dxi * (r - g.r0);
  const double s = t.s[o2][j + g.ng], c = t.c[o2][j + g.ng];
  const double T = g.h0 == 0.0 ? g.dth : t.td[o2][j + g.ng];
  const double a2 = g.a * g.a, r2 = r * r, tMr = 2.0 * g.M * r;
  const double Sig = r2 + a2 * c * c;
  const double S2 = Sig + tMr;
  const double ra = r2 + a2;
  const double A = ra * ra - a2 * (ra - tMr) * s * s;
  const double opz = S2 / Sig;
  Cell e;
  e.alpha = sqrt(Sig / S2);
  e.beta1 = tMr / (S2 * R);
  e.hl11 = opz * R * R;
  e.hl22 = Sig * T * T;
  e.hl33 = A * s * s / Sig;
  e.hl13 = -g.a * opz * s * s * R;
  e.sqrt_ht = R * T * Sig / e.alpha;
  e.sqrt_h = e.sqrt_ht * s;
  return e;
}

// ---------------------------------------------------------------- weights
// Solver weights at one staggered point (i + o1/2, j + o2/2).  With
// S2 = Sigma + 2 M r and k = 1/sqrt(Sigma S2), the lapse is Sigma k,
// 1/Sigma = S2 k^2, 1/S2 = Sigma k^2 and sqrt(h)/sin(theta) = R T / k
// (R = dr/dx1, T = dtheta/dx2), so one reciprocal square root gives every factor of the
// closed forms of App. A (the same quantities as cell_tab).
struct FW {
  double alpha;                   // lapse
  double hl11, hl22, hl33;        // lower spatial metric, code components
  double w13;                     // sqrt(h)/sin * h_13       (radial-average weight)
  double wb;                      // sqrt(h)/sin * sqrt(h) * beta^1
  double h_sht;                   // 1 / (2 sqrt(h)/sin)      (radial-average norm)
  double ish;                     // 1 / sqrt(h)              (0 on the axis)
};

// kQ: the general quasi-spherical map (r0, h0 not both 0); otherwise the
// logarithmic-r, uniform-theta grid, with R = dxi r and T = deta.
template <bool kQ>
__device__ inline FW fw_tab(const Grid& g, const Tables& t, int i, int o1, int j, int o2) {
  const double r = t.r[o1][i + g.ng], R = g.dxi * (kQ ? r - g.r0 : r);
  const double s = t.s[o2][j + g.ng], c = t.c[o2][j + g.ng], is = t.is[o2][j + g.ng];
  const double T = kQ ? t.td[o2][j + g.ng] : g.dth;
  const double ird = kQ ? t.ird[o1][i + g.ng] * t.eta_t[o2][j + g.ng] : t.ird[o1][i + g.ng];  // 1/(R T)
  const double a2 = g.a * g.a, r2 = r * r, tMr = 2.0 * g.M * r, s2 = s * s;
  const double Sig = r2 + a2 * c * c;
  const double S2 = Sig + tMr;
  const double ra = r2 + a2;
  const double A = ra * ra - a2 * (ra - tMr) * s2;
  const double k = rsqrt(Sig * S2);
  const double k2 = k * k;
  const double S2k = S2 * k;
  FW e;
  e.alpha = Sig * k;
  e.hl11 = S2k * S2k * R * R;
  e.hl22 = Sig * T * T;
  e.hl33 = A * s2 * S2 * k2;
  e.w13 = -g.a * T * R * R * s2 * S2 * S2k;
  e.wb = R * T * T * s * tMr * Sig;
  e.h_sht = 0.5 * k * ird;
  e.ish = k * ird * is;
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

// Whole-plane thread index (ghosts included): j along theta, i along r.
struct PlaneIdx {
  int i, j;
  bool ok;
};
__device__ inline PlaneIdx plane_idx(const Grid& g) {
  PlaneIdx q;
  q.j = (int)(blockIdx.x * blockDim.x + threadIdx.x) - g.ng;
  q.i = (int)(blockIdx.y * blockDim.y + threadIdx.y) - g.ng;
  q.ok = q.j < g.n_th + g.ng && q.i < g.n_r + g.ng;
  return q;
}

// ---------------------------------------------------------------- aux E, H
// eq. discretized-auxE/-auxH with the volume-weighted radial averages of
// Sec. 3.3.1 (weights sqrt(h)/sin(theta)); for i in [-1, n_r], j in [0, n_th].
// kE / kH select the outputs; both read the same B, D and share the weights.
template <class T, bool kE, bool kH, bool kQ>
__global__ void aux_kernel(Grid g, Tables t, CTriT<T> Bs, CTriT<T> Ds, TriT<T> E, TriT<T> H) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y - 1;
  if (j > g.n_th || i > g.n_r) return;
  const int64_t o = ix(g, i, j), ld = g.ld;
  const bool half = j < g.n_th;  // theta-staggered components exist
  // weights at the points the stencils touch (unused ones are not computed)
  const FW n00 = fw_tab<kQ>(g, t, i, 0, j, 0);       // (i, j)
  const FW n10 = fw_tab<kQ>(g, t, i + 1, 0, j, 0);   // (i+1, j)
  const FW h00 = fw_tab<kQ>(g, t, i, 1, j, 0);       // (i+1/2, j)
  const FW hm0 = fw_tab<kQ>(g, t, i - 1, 1, j, 0);   // (i-1/2, j)
  const FW n01 = fw_tab<kQ>(g, t, i, 0, j, 1);       // (i, j+1/2)
  const FW n11 = fw_tab<kQ>(g, t, i + 1, 0, j, 1);   // (i+1, j+1/2)
  const FW h01 = fw_tab<kQ>(g, t, i, 1, j, 1);       // (i+1/2, j+1/2)
  const FW hm1 = fw_tab<kQ>(g, t, i - 1, 1, j, 1);   // (i-1/2, j+1/2)
  if (kE) {
    {  // E_1 (i+1/2, j)
      const double av = (n00.w13 * Ds.p[2][o] + n10.w13 * Ds.p[2][o + ld]) * h00.h_sht;
      E.p[0][o] = h00.alpha * (h00.hl11 * Ds.p[0][o] + av);
    }
    {  // E_3 (i, j)
      const double a1 = (hm0.w13 * Ds.p[0][o - ld] + h00.w13 * Ds.p[0][o]) * n00.h_sht;
      const double a2 = (hm0.wb * Bs.p[1][o - ld] + h00.wb * Bs.p[1][o]) * n00.h_sht;
      E.p[2][o] = n00.alpha * (n00.hl33 * Ds.p[2][o] + a1) + a2;
    }
    if (half) {  // E_2 (i, j+1/2)
      const double a3 = (hm1.wb * Bs.p[2][o - ld] + h01.wb * Bs.p[2][o]) * n01.h_sht;
      E.p[1][o] = n01.alpha * n01.hl22 * Ds.p[1][o] - a3;
    }
  }
  if (kH) {
    {  // H_2 (i+1/2, j)
      const double a1 = (n00.wb * Ds.p[2][o] + n10.wb * Ds.p[2][o + ld]) * h00.h_sht;
      H.p[1][o] = h00.alpha * h00.hl22 * Bs.p[1][o] + a1;
    }
    if (half) {
      {  // H_1 (i, j+1/2)
        const double a2 = (hm1.w13 * Bs.p[2][o - ld] + h01.w13 * Bs.p[2][o]) * n01.h_sht;
        H.p[0][o] = n01.alpha * (n01.hl11 * Bs.p[0][o] + a2);
      }
      {  // H_3 (i+1/2, j+1/2)
        const double a3 = (n01.w13 * Bs.p[0][o] + n11.w13 * Bs.p[0][o + ld]) * h01.h_sht;
        const double a4 = (n01.wb * Ds.p[1][o] + n11.wb * Ds.p[1][o + ld]) * h01.h_sht;
        H.p[2][o] = h01.alpha * (h01.hl33 * Bs.p[2][o] + a3) - a4;
      }
    }
  }
}

// ---------------------------------------------------------------- Faraday
// eq. discretized-faraday on the evolved ranges i in [0, n_r], j in [0, n_th].
// With kSave the grid spans the whole plane and X0 <- X (the field before the
// update, ghosts included) is taken in the same pass.
template <class T, bool kSave, bool kQ>
__global__ void faraday_kernel(Grid g, Tables t, TriT<T> X, TriT<T> L, CTriT<T> E, TriT<T> X0) {
  int i, j;
  if (kSave) {
    const PlaneIdx q = plane_idx(g);
    if (!q.ok) return;
    i = q.i;
    j = q.j;
  } else {
    j = blockIdx.x * blockDim.x + threadIdx.x;
    i = blockIdx.y * blockDim.y + threadIdx.y;
  }
  const int64_t o = ix(g, i, j);
  if (kSave) {
#pragma unroll
    for (int c = 0; c < 3; ++c) X0.p[c][o] = X.p[c][o];
  }
  if (i < 0 || j < 0 || j > g.n_th || i > g.n_r) return;
  if (j < g.n_th) {
    const double ish = fw_tab<kQ>(g, t, i, 0, j, 1).ish;
    add_to(X.p[0], L.p[0], o, -(g.dt * (E.p[2][o + 1] - E.p[2][o]) * ish));
  }
  if (i < g.n_r && j >= 1 && j < g.n_th) {
    const double ish = fw_tab<kQ>(g, t, i, 1, j, 0).ish;
    add_to(X.p[1], L.p[1], o, g.dt * (E.p[2][o + g.ld] - E.p[2][o]) * ish);
  }
  if (i < g.n_r && j < g.n_th) {
    const double ish = fw_tab<kQ>(g, t, i, 1, j, 1).ish;
    const double curl = (E.p[1][o + g.ld] - E.p[1][o]) - (E.p[0][o + 1] - E.p[0][o]);
    add_to(X.p[2], L.p[2], o, -(g.dt * curl * ish));
  }
}

// ---------------------------------------------------------------- Ampere
// eq. discretized-ampere with the current J = wa Ja + wb Jb; D^1 on the axis
// rows from the polar-cap integral form (Sec. 3.3.2): cap area A_{i+1/2}, the
// printed 2 pi with the two-sided (mirrored) axis-row current the deposit
// leaves there; the theta = pi cap has the opposite orientation.
// kFinal (the last half of the step): the grid spans the whole plane, the
// current is Ja alone, and the same pass takes X0 <- X before the update and
// rotates the currents after it: Jb <- Ja, and the deposit's accumulator is
// zeroed (Jclear, or Ja itself when Jclear is null: the filter leaves the
// filtered current in the scratch set or in the accumulator).
template <class T, bool kFinal, bool kQ>
__global__ void ampere_kernel(Grid g, Tables t, TriT<T> X, TriT<T> L, CTriT<T> H, TriT<T> Ja, TriT<T> Jb, double wa,
                              double wb, double polar_k, TriT<T> X0, TriT<T> Jclear) {
  int i, j;
  if (kFinal) {
    const PlaneIdx q = plane_idx(g);
    if (!q.ok) return;
    i = q.i;
    j = q.j;
  } else {
    j = blockIdx.x * blockDim.x + threadIdx.x;
    i = blockIdx.y * blockDim.y + threadIdx.y;
  }
  const int64_t o = ix(g, i, j);
  if (kFinal) {
#pragma unroll
    for (int c = 0; c < 3; ++c) X0.p[c][o] = X.p[c][o];
  }
  if (!(i < 0 || j < 0 || j > g.n_th || i > g.n_r)) {
    const double fpi = 4.0 * kPi;
    auto cur = [&](int c) -> double {
      return kFinal ? (double)Ja.p[c][o] : wa * Ja.p[c][o] + wb * Jb.p[c][o];
    };
    if (i < g.n_r) {
      const double J1 = cur(0);
      if (j >= 1 && j < g.n_th) {
        const double ish = fw_tab<kQ>(g, t, i, 1, j, 0).ish;
        add_to(X.p[0], L.p[0], o, g.dt * ((H.p[2][o] - H.p[2][o - 1]) - fpi * J1) * ish);
      } else {
        const double r = t.r[1][i + g.ng];
        const double ra = r * r + g.a * g.a;
        const double Ap = g.dxi * (kQ ? r - g.r0 : r) * ra * sqrt(1.0 + 2.0 * g.M * r / ra) * polar_k;
        const double h3 = (j == 0) ? H.p[2][o] : -H.p[2][o - 1];
        add_to(X.p[0], L.p[0], o, g.dt * (h3 - 2.0 * kPi * J1) / Ap);
      }
    }
    if (j < g.n_th) {
      const double ish = fw_tab<kQ>(g, t, i, 0, j, 1).ish;
      const double J2 = cur(1);
      add_to(X.p[1], L.p[1], o, g.dt * (-(H.p[2][o] - H.p[2][o - g.ld]) - fpi * J2) * ish);
    }
    if (j >= 1 && j < g.n_th) {
      const double ish = fw_tab<kQ>(g, t, i, 0, j, 0).ish;
      const double J3 = cur(2);
      const double curl = (H.p[1][o] - H.p[1][o - g.ld]) - (H.p[0][o] - H.p[0][o - 1]);
      add_to(X.p[2], L.p[2], o, g.dt * (curl - fpi * J3) * ish);
    }
  }
  if (kFinal) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Jb.p[c][o] = Ja.p[c][o];
      (Jclear.p[0] ? Jclear.p[c] : Ja.p[c])[o] = 0.0;
    }
  }
}

// ---------------------------------------------------------------- boundaries
// One block per plane row i in [-ng, n_r + ng - 1], the radial conditions
// first, then the axis:
//  - constant layer inside the horizon (rows i <= n_f take row n_f + 1) and
//    the absorbing layer (F <- F - lambda (F - F_init), lambda a cubic ramp
//    over the last n_absorb cells), on every column;  half1[c] = staggering of
//    component c in x1;
//  - axis reflection (Sec. 3.3.3): r-components even, theta and phi
//    components odd, ghost columns from the row's own updated values; with
//    zero_comp, the theta component of B (B^2) or the phi component of D (D^3)
//    vanishes on the axis rows.  half2[c] = staggering in x2.
// Rows i <= n_f read row n_f + 1, which neither layer changes; the axis pass of
// that row may run first and only rewrites entries that each row's own axis
// pass rewrites again.
// With radial = 0 only the axis reflection is applied (initial data).
template <class T>
__global__ void bc_kernel(Grid g, TriT<T> X, TriT<T> L, CTriT<T> X0, int3 half1, int3 half2, int zero_comp,
                          int radial) {
  const int i = (int)blockIdx.x - g.ng;
  const int h1[3] = {half1.x, half1.y, half1.z};
  const int h2[3] = {half2.x, half2.y, half2.z};
  const bool comp = sizeof(T) == 4 && L.p[0];
  const bool horizon = i <= g.n_filter;
  const double x0 = (double)(g.n_r - g.n_absorb);
  if (radial && (horizon || (g.n_absorb > 0 && (double)i + 0.5 > x0))) {
    for (int j = (int)threadIdx.x - g.ng; j < g.n_th + g.ng; j += blockDim.x) {
      const int64_t o = ix(g, i, j);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (horizon) {
          const int64_t src = ix(g, g.n_filter + 1, j);
          X.p[c][o] = X.p[c][src];
          if (comp) L.p[c][o] = L.p[c][src];
        } else {
          const double x = (double)i + 0.5 * h1[c];
          if (x > x0) {
            const double sr = fmin((x - x0) / g.n_absorb, 1.0);
            const double lam = sr * sr * sr;
            if (comp) {
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
  }
  __syncthreads();
  // one lane per (component, ghost column): the 2 ng ghost columns of each
  // component, each the reflection of its mirror column (node rows run 0..n,
  // half rows 0..n-1); the mirrors are interior columns, which this pass only
  // zeroes at j = 0, n for zero_comp, and never reads
  const int t = threadIdx.x;
  if (t >= 3 * 2 * g.ng) return;
  const int c = t / (2 * g.ng), q = t % (2 * g.ng);
  const int n = g.n_th;
  T* C = X.p[c];
  const int j = q < g.ng ? -1 - q : n - h2[c] + 1 + (q - g.ng);  // ghost column
  const bool exists = j < n + g.ng;
  const int m = j < 0 ? (h2[c] ? -1 - j : -j) : (h2[c] ? 2 * n - 1 - j : 2 * n - j);
  const T v = exists ? C[ix(g, i, m)] : (T)0;
  if (exists) C[ix(g, i, j)] = (c == 0 ? 1.0 : -1.0) * v;
  if (!h2[c] && c == zero_comp && (q == 0 || q == g.ng)) {
    const int jz = q == 0 ? 0 : n;
    C[ix(g, i, jz)] = 0.0;
    if (comp) L.p[c][ix(g, i, jz)] = 0.0;
  }
}

// ---------------------------------------------------------------- misc
// elementwise over whole planes (ghosts included)
template <class T>
__global__ void average_kernel(int64_t n, TriT<T> A, CTriT<T> B, TriT<T> C, CTriT<T> D) {
  // A <- (A + B) / 2, C <- (C + D) / 2
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    A.p[c][k] = 0.5 * (A.p[c][k] + B.p[c][k]);
    C.p[c][k] = 0.5 * (C.p[c][k] + D.p[c][k]);
  }
}

template <class T>
__global__ void copy_kernel(int64_t n, TriT<T> A, CTriT<T> B) {  // A <- B
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) A.p[c][k] = B.p[c][k];
}

template <class T>
__global__ void fill_kernel(int64_t n, T* __restrict__ p, double v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// Column j reflected across the axis for a component of x2-staggering hs
// (node rows run 0..n, half rows 0..n-1); interior columns map to themselves.
__device__ inline int axis_mirror(int j, int n, int hs) {
  if (j < 0) return hs ? -1 - j : -j;
  if (j > n - hs) return hs ? 2 * n - 1 - j : 2 * n - j;
  return j;
}

// The value one binomial pass (1,2,1)/4 x (1,2,1)/4 (Sec. 3.3.4) gives at
// plane point (i, j) of a component of x2-staggering hs and axis parity par,
// from the source values at(i', j'): ghost columns take the source's axis
// reflection, the two outermost rows keep the source, every other point is
// the stencil with its theta neighbours read as axis reflections where they
// fall past an axis (so at() is only asked for evolved columns there).
template <class T, class At>
__device__ inline T filter_point(const Grid& g, int i, int j, int hs, double par, const At& at) {
  const int n = g.n_th;
  if (j < 0 || j > n - hs) return (T)(par * (double)at(i, axis_mirror(j, n, hs)));
  if (i < 1 - g.ng || i > g.n_r + g.ng - 2) return at(i, j);
  const int jm = axis_mirror(j - 1, n, hs), jp = axis_mirror(j + 1, n, hs);
  const double pm = jm == j - 1 ? 1.0 : par, pp = jp == j + 1 ? 1.0 : par;
  const double r0 = pm * (double)at(i - 1, jm) + 2.0 * (double)at(i - 1, j) + pp * (double)at(i - 1, jp);
  const double r1 = pm * (double)at(i, jm) + 2.0 * (double)at(i, j) + pp * (double)at(i, jp);
  const double r2 = pm * (double)at(i + 1, jm) + 2.0 * (double)at(i + 1, j) + pp * (double)at(i + 1, jp);
  return (T)(0.0625 * (r0 + 2.0 * r1 + r2));
}

// One binomial pass of S into X over the whole plane (filter_point per
// point).  Passes alternate between two plane sets.
template <class T>
__global__ void filter_kernel(Grid g, TriT<T> X, CTriT<T> S, int3 half2, int3 parity, int ncomp) {
  const PlaneIdx q = plane_idx(g);
  if (!q.ok) return;
  const int hs[3] = {half2.x, half2.y, half2.z};
  const int ps[3] = {parity.x, parity.y, parity.z};
  const int64_t o = ix(g, q.i, q.j);
  for (int c = 0; c < ncomp; ++c) {
    const T* s = S.p[c];
    auto at = [&](int i, int j) -> T { return s[ix(g, i, j)]; };
    X.p[c][o] = filter_point<T>(g, q.i, q.j, hs[c], (double)ps[c], at);
  }
}

// Up to kFMaxPasses binomial passes of S into X in one launch.  A block
// (64 x 4 threads) owns an output tile of kFTI rows x kFTJ plane columns and
// stages it in LDS with a halo as wide as the number of passes (and, at the
// far axis, the columns its ghost columns reflect).  Each pass runs in two
// LDS sweeps, the theta sums of every row (pm S[j-1] + 2 S[j] + pp S[j+1],
// FP64), then the radial combination (R[i-1] + 2 R[i] + R[i+1]) / 16 rounded
// to T, exactly the arithmetic of filter_point; ghost columns take the axis
// reflection and the two outermost plane rows are copied.  Points whose
// neighbours lie outside the staged region are not computed: the stale values
// at the region's edge move inwards by one point per pass, so after `passes`
// passes the tile (at depth `passes`) is exact; at the plane's edges nothing
// outside is needed.  X must not alias S (other blocks read S's halo).
// n_ghost = 2.
constexpr int kFTI = 32, kFTJ = 48, kFMaxPasses = 4;
constexpr int kFLI = kFTI + 2 * kFMaxPasses, kFLJ = 64;  // kFTJ + 2 passes + 6 far-axis columns <= 64

template <class T>
__global__ void __launch_bounds__(256) filter_fused_kernel(Grid g, TriT<T> X, CTriT<T> S, int3 half2,
                                                           int3 parity, int ncomp, int passes) {
  __shared__ T buf[2][kFLI][kFLJ];
  __shared__ double rs[kFLI][kFLJ];
  const int hs3[3] = {half2.x, half2.y, half2.z};
  const int ps3[3] = {parity.x, parity.y, parity.z};
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int n = g.n_th;
  const int i0 = (int)blockIdx.y * kFTI - g.ng;  // first output row (plane row index i)
  const int J0 = (int)blockIdx.x * kFTJ;         // first output column (storage column, j + ng)
  const int far = J0 + kFTJ > n + g.ng - 4 ? 2 * g.ng + 2 : 0;
  const int ilo = max(i0 - passes, -g.ng), ihi = min(i0 + kFTI + passes, g.n_r + g.ng);
  const int Jlo = max(J0 - passes - far, 0), Jhi = min(J0 + kFTJ + passes, g.ld);
  const int ni = ihi - ilo, nj = Jhi - Jlo;
  const int j = Jlo + tx - g.ng;  // this thread's plane column
  for (int c = 0; c < ncomp; ++c) {
    const int hs = hs3[c];
    const double par = (double)ps3[c];
    const bool ghost = j < 0 || j > n - hs;
    // LDS columns this thread reads: the axis reflection (ghost column) or
    // the two theta neighbours with their parities
    const int jr = axis_mirror(j, n, hs) + g.ng - Jlo;
    const int jm = axis_mirror(j - 1, n, hs), jp = axis_mirror(j + 1, n, hs);
    const double pm = jm == j - 1 ? 1.0 : par, pp = jp == j + 1 ? 1.0 : par;
    const int lm = jm + g.ng - Jlo, lp = jp + g.ng - Jlo;
    const bool col = tx < nj;
    const bool sums = col && !ghost && lm >= 0 && lm < nj && lp >= 0 && lp < nj;
    const bool refl = col && ghost && jr >= 0 && jr < nj;
    const T* s = S.p[c];
    if (col)
      for (int li = ty; li < ni; li += 4) buf[0][li][tx] = s[(int64_t)(ilo + li + g.ng) * g.ld + (Jlo + tx)];
    __syncthreads();
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
      if (sums)
        for (int li = ty; li < ni; li += 4)
          rs[li][tx] = pm * (double)buf[cur][li][lm] + 2.0 * (double)buf[cur][li][tx] + pp * (double)buf[cur][li][lp];
      __syncthreads();
      if (col)
        for (int li = ty; li < ni; li += 4) {
          const int i = ilo + li;
          T v;
          if (ghost) {
            if (!refl) continue;
            v = (T)(par * (double)buf[cur][li][jr]);
          } else if (i < 1 - g.ng || i > g.n_r + g.ng - 2) {
            v = buf[cur][li][tx];
          } else {
            if (li == 0 || li == ni - 1) continue;  // the staged region's edge: neighbours not staged
            v = (T)(0.0625 * (rs[li - 1][tx] + 2.0 * rs[li][tx] + rs[li + 1][tx]));
          }
          buf[cur ^ 1][li][tx] = v;
        }
      __syncthreads();
      cur ^= 1;
    }
    T* x = X.p[c];
    const int J = Jlo + tx;
    if (col && J >= J0 && J < J0 + kFTJ)
      for (int li = ty; li < ni; li += 4) {
        const int i = ilo + li;
        if (i >= i0 && i < i0 + kFTI) x[(int64_t)(i + g.ng) * g.ld + J] = buf[cur][li][tx];
      }
    __syncthreads();
  }
}

}  // namespace grpic
