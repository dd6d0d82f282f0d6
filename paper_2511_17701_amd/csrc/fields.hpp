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
// The radial conditions (bc_radial_kernel), then the axis (bc_axis_kernel):
//  - constant layer inside the horizon (rows i <= n_f take row n_f + 1) and
//    the absorbing layer (F <- F - lambda (F - F_init), lambda a cubic ramp
//    over the last n_absorb cells), on every column;  half1[c] = staggering of
//    component c in x1;
//  - axis reflection (Sec. 3.3.3): r-components even, theta and phi
//    components odd, ghost columns from the row's updated values; with
//    zero_comp, the theta component of B (B^2) or the phi component of D (D^3)
//    vanishes on the axis rows.  half2[c] = staggering in x2.
// Rows i <= n_f read row n_f + 1, which neither layer changes.  Initial data
// take only the axis reflection.

// Rows of the two layers: the horizon rows [-ng, n_f] and the absorbing rows
// [abs_begin, n_r + ng) (a row in both is a horizon row).
struct BcRows {
  int n_hor, n_abs;  // number of horizon / absorbing rows
  int abs_begin;     // first absorbing row
};

__host__ __device__ inline BcRows bc_rows(const Grid& g) {
  BcRows b;
  const int top = g.n_r + g.ng;                  // one past the last plane row
  const int hor_end = min(g.n_filter + 1, top);  // horizon rows: i <= n_f
  b.abs_begin = g.n_absorb > 0 ? max(hor_end, g.n_r - g.n_absorb) : top;
  b.n_hor = hor_end + g.ng;
  b.n_abs = top - b.abs_begin;
  return b;
}

// One thread per (layer row, stored column): grid (ceil(ld / 256), n_hor +
// n_abs), 256 threads.
template <class T>
__global__ void bc_radial_kernel(Grid g, TriT<T> X, TriT<T> L, CTriT<T> X0, int3 half1) {
  const BcRows rows = bc_rows(g);
  const int r = (int)blockIdx.y;
  const bool horizon = r < rows.n_hor;
  const int i = horizon ? r - g.ng : rows.abs_begin + (r - rows.n_hor);
  const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x) - g.ng;
  if (j >= g.n_th + g.ng) return;
  const int h1[3] = {half1.x, half1.y, half1.z};
  const bool comp = sizeof(T) == 4 && L.p[0];
  const double x0 = (double)(g.n_r - g.n_absorb);
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

// 6 ng lanes per plane row, one per (component, ghost column): bc_axis_rows
// rows per block of `threads`.
__host__ __device__ inline int bc_axis_rows(const Grid& g, int threads) { return threads / (6 * g.ng); }

// Axis reflection of every plane row: each ghost column of a component is
// the reflection of its mirror column (node rows run 0..n, half rows
// 0..n-1); the mirrors are interior columns, which this pass only zeroes at
// j = 0, n for zero_comp, and never reads.
template <class T>
__global__ void bc_axis_kernel(Grid g, TriT<T> X, TriT<T> L, int3 half2, int zero_comp) {
  const int lanes = 6 * g.ng, rpb = bc_axis_rows(g, (int)blockDim.x);
  const int t = (int)threadIdx.x;
  const int i = (int)blockIdx.x * rpb + t / lanes - g.ng;
  if (t >= rpb * lanes || i >= g.n_r + g.ng) return;
  const int h2[3] = {half2.x, half2.y, half2.z};
  const bool comp = sizeof(T) == 4 && L.p[0];
  const int c = (t % lanes) / (2 * g.ng), q = (t % lanes) % (2 * g.ng);
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

// ---------------------------------------------------------------- filter
// Binomial passes (1,2,1)/4 x (1,2,1)/4 of a current plane (Sec. 3.3.4), in
// the arithmetic of one pass at plane point (i, j) of a component of
// x2-staggering hs and axis parity par, reading the source S of the pass:
//  - ghost columns (j < 0 or j > n_th - hs) take the source's axis reflection
//    par S(i, mirror(j));
//  - the two outermost plane rows keep the source;
//  - every other point is (R(i-1) + 2 R(i) + R(i+1)) / 16 rounded to T, with
//    the FP64 row sums R(i) = pm S(i, j-1) + 2 S(i, j) + pp S(i, j+1), whose
//    theta neighbours past an axis are read as reflections (pm, pp = par
//    there, 1 elsewhere).
// Every product is by 1, 2 or a power of two, so the result does not depend
// on how the compiler contracts the sums.
//
// Up to kFMaxPasses passes run in one launch.  A wavefront owns a strip of
// 64 plane columns (one per lane) and kSR output rows, and holds its rows plus
// a halo of P rows on each side in registers for the whole run: the theta
// neighbours come from the adjacent lanes by DPP wave shifts and the axis
// reflections by a lane permute (only in strips that touch an axis); the
// radial sums slide down the rows.  No LDS and no barriers.  Values whose
// neighbours lie outside the strip (the wave's first and last lane, the first
// and last staged row) are not computed: the stale points move inwards by one
// per pass, so after P passes the 56 middle lanes and the kSR middle rows are
// exact; at the plane's edges nothing outside is needed and the strip outputs
// up to the edge.  The last strip of a row is shifted to end at the plane's
// last column, so the far-axis reflections it reads are exact (the columns it
// shares with its neighbour get identical values twice).  X must not alias S.
constexpr int kFMaxPasses = 4;
constexpr int kFLanes = 64, kFOut = kFLanes - 2 * kFMaxPasses;  // 56 output columns per strip

// number of 64-column strips that cover a plane row of ld stored columns,
// and the first stored column of strip b (the last one ends at the plane's
// last column)
__host__ __device__ inline int filter_strips_theta(int ld) {
  return ld <= kFLanes ? 1 : (ld - (kFLanes - kFMaxPasses) + kFOut - 1) / kFOut + 1;
}
__host__ __device__ inline int filter_strip_lo(int b, int ld) {
  return min(b * kFOut, max(ld - kFLanes, 0));
}
// whether strip b touches an axis (a column j <= 0 or j >= n_th - 1)
__host__ __device__ inline bool filter_strip_axis(int b, int ld, int n, int ng) {
  const int lo = filter_strip_lo(b, ld);
  return lo <= ng || lo + kFLanes - 1 >= n - 1 + ng;
}

// the lane's value one lane down (wave_shr:1) and one lane up (wave_shl:1);
// the first / last lane reads 0
__device__ inline int lane_down(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false); }
__device__ inline int lane_up(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false); }
__device__ inline float lane_down(float v) { return __int_as_float(lane_down(__float_as_int(v))); }
__device__ inline float lane_up(float v) { return __int_as_float(lane_up(__float_as_int(v))); }
__device__ inline double lane_down(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_down((int)(b & 0xffffffffll)), hi = lane_down((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
__device__ inline double lane_up(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_up((int)(b & 0xffffffffll)), hi = lane_up((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// Column j reflected across the axis for a component of x2-staggering hs
// (node rows run 0..n, half rows 0..n-1); interior columns map to themselves.
__device__ inline int axis_mirror(int j, int n, int hs) {
  if (j < 0) return hs ? -1 - j : -j;
  if (j > n - hs) return hs ? 2 * n - 1 - j : 2 * n - j;
  return j;
}

// Lane-constant data of one component in a strip that touches an axis.
struct FilterAxis {
  bool lo, hi;     // j == 0 / j == n - hs: the theta neighbour past the axis is a reflection
  bool ghost;      // ghost column
  int src;         // lane of the reflected column (ghost lanes)
  bool hs;         // half-staggered in x2
  double par;      // axis parity
};

// FP64 theta row sum of the pass at this lane
template <class T, bool kAxis>
__device__ inline double filter_row_sum(T a, const FilterAxis& ax) {
  const T dn = lane_down(a), up = lane_up(a);
  double lv = (double)dn, rv = (double)up;
  if (kAxis) {
    if (ax.lo) lv = ax.par * (double)(ax.hs ? a : up);
    if (ax.hi) rv = ax.par * (double)(ax.hs ? a : dn);
  }
  return (lv + 2.0 * (double)a) + rv;
}

// One component of a strip: load, P passes, store rows [rlo, rhi).  kAxis:
// the strip touches an axis (reflected neighbours, ghost columns); kRows: a
// plane of fewer rows than a strip stages (rows outside the plane, the two
// kept rows inside the strip).  Otherwise the strips are placed so that the
// kept rows are a strip's first or last staged row, which no pass updates.
template <class T, int P, int kSR, bool kAxis, bool kRows>
__device__ __forceinline__ void filter_strip_comp(const Grid& g, T* __restrict__ x, const T* __restrict__ s,
                                                  int J, bool col, bool out, int ifirst, int rlo, int rhi,
                                                  const FilterAxis& ax) {
  constexpr int R = kSR + 2 * P;
  // one wavefront-uniform base (the strip's first staged row) and 32-bit
  // per-lane byte offsets (a strip spans R rows: far below 4 GiB)
  const int64_t row0 = (int64_t)(ifirst + g.ng) * g.ld;
  const char* __restrict__ sb = (const char*)(s + row0);
  const uint32_t rowb = (uint32_t)(g.ld * sizeof(T)), lb = (uint32_t)(J * sizeof(T));
  T v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ifirst + r;
    v[r] = col && (!kRows || (i >= -g.ng && i < g.n_r + g.ng)) ? *(const T*)(sb + (lb + (uint32_t)r * rowb))
                                                                : (T)0;
    if ((r & 7) == 7) __builtin_amdgcn_sched_barrier(0);  // 8 row offsets live at a time
  }
#pragma unroll 1
  for (int p = 0; p < P; ++p) {
    double s_prev = 0.0, s_cur = filter_row_sum<T, kAxis>(v[0], ax);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double s_next = r + 1 < R ? filter_row_sum<T, kAxis>(v[r + 1], ax) : 0.0;
      const int i = ifirst + r;
      T nv = v[r];
      if (r >= 1 && r <= R - 2 && (!kRows || (i >= 1 - g.ng && i <= g.n_r + g.ng - 2)))
        nv = (T)(0.0625 * ((s_prev + 2.0 * s_cur) + s_next));
      if (kAxis) {
        const T m = __shfl(v[r], ax.src);
        if (ax.ghost) nv = (T)(ax.par * (double)m);
      }
      v[r] = nv;
      s_prev = s_cur;
      s_cur = s_next;
      __builtin_amdgcn_sched_barrier(0);  // row by row: a few sums live, not all
    }
  }
  if (out) {
    // an opaque copy of the lane offset: the stores recompute their row
    // offsets instead of keeping the loads' live through the passes
    uint32_t lbs = lb;
    asm volatile("" : "+v"(lbs));
    char* __restrict__ db = (char*)(x + row0);
    auto put = [&](int r) { *(T*)(db + (lbs + (uint32_t)r * rowb)) = v[r]; };
    if (kRows) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (r >= rlo && r < rhi && ifirst + r < g.n_r + g.ng) put(r);
    } else {  // rows [rlo, rhi) = [P or 0, P + kSR or R)
#pragma unroll
      for (int r = P; r < P + kSR; ++r) put(r);
      if (rlo == 0) {
#pragma unroll
        for (int r = 0; r < P; ++r) put(r);
      }
      if (rhi == R) {
#pragma unroll
        for (int r = P + kSR; r < R; ++r) put(r);
      }
    }
  }
}

// number of row strips of a plane with nrow rows (kRows: nrow < kSR + 2 P)
template <int P, int kSR, bool kRows>
__host__ __device__ inline int filter_strips_r(int nrow) {
  return kRows ? (nrow + kSR - 1) / kSR : (nrow - (kSR + 2 * P) + kSR - 1) / kSR + 1;
}

// P passes of S into X, plane blockIdx.z.  Grid: (filter_strips_theta(ld),
// ceil(filter_strips_r / 4), number of planes); 256 threads = 4 wavefronts on
// consecutive row strips.  Strip s stages rows from min(s kSR - ng,
// n_r + ng - R) (kRows: s kSR - ng - P) and writes the rows it has exact:
// from its first row in the first strip, to its last in the last one.  The register budget (four
// wavefronts per SIMD, two for a single pass) keeps the compiler from
// computing every row sum of a pass ahead of the radial combinations.
template <class T, int P, int kSR, bool kRows>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == 1 ? 2 : 4)))
filter_strip_kernel(Grid g, TriT<T> X, CTriT<T> S, int3 half2, int3 parity) {
  constexpr int R = kSR + 2 * P;
  const int lane = (int)threadIdx.x & (kFLanes - 1);
  const int strip = (int)blockIdx.y * 4 + ((int)threadIdx.x >> 6);
  const int nrow = g.n_r + 2 * g.ng;
  if (strip >= filter_strips_r<P, kSR, kRows>(nrow)) return;  // whole wavefront
  int ifirst, rlo, rhi;
  if (kRows) {
    ifirst = strip * kSR - g.ng - P;
    rlo = P;
    rhi = P + kSR;
  } else {
    ifirst = min(strip * kSR - g.ng, g.n_r + g.ng - R);
    rlo = strip == 0 ? 0 : P;
    rhi = ifirst + R >= g.n_r + g.ng ? R : P + kSR;
  }
  const int ld = (int)g.ld, n = g.n_th;
  const int b = (int)blockIdx.x;
  const int Jlo = filter_strip_lo(b, ld);
  const int out_lo = b == 0 ? 0 : Jlo + kFMaxPasses;
  const int out_hi = Jlo + kFLanes >= ld ? ld : Jlo + kFLanes - kFMaxPasses;
  const int J = Jlo + lane, j = J - g.ng;
  const bool col = J < ld, out = col && J >= out_lo && J < out_hi;
  // one component per grid.z (plane pointers selected with scalar code)
  const int c = (int)blockIdx.z;
  const int hs = c == 0 ? half2.x : c == 1 ? half2.y : half2.z;
  T* const x = c == 0 ? X.p[0] : c == 1 ? X.p[1] : X.p[2];
  const T* const sp = c == 0 ? S.p[0] : c == 1 ? S.p[1] : S.p[2];
  FilterAxis ax{};
  const bool axis = filter_strip_axis(b, ld, n, g.ng);  // whole wavefront
  if (axis) {
    ax.hs = hs != 0;
    ax.par = (double)(c == 0 ? parity.x : c == 1 ? parity.y : parity.z);
    ax.lo = j == 0;
    ax.hi = j == n - hs;
    ax.ghost = j < 0 || j > n - hs;
    ax.src = ax.ghost ? lane + axis_mirror(j, n, hs) - j : lane;
  }
  if (axis)
    filter_strip_comp<T, P, kSR, true, kRows>(g, x, sp, J, col, out, ifirst, rlo, rhi, ax);
  else
    filter_strip_comp<T, P, kSR, false, kRows>(g, x, sp, J, col, out, ifirst, rlo, rhi, ax);
}

}  // namespace grpic
