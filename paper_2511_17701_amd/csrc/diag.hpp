// diag.hpp -- diagnostics kernels: conserved energy / angular momentum per
// particle (Sec. 2.3), slot counts, and the Gauss-law residual (Sec. 3.2).
#pragma once

#include "init.hpp"

namespace grpic {

// Device accumulators: counts[0..3] alive by species, [4] leaving, [5] empty,
// [6] non-finite; sums[0..3] E by species, [4..7] L by species; the two maxima
// are non-negative doubles compared through their bit patterns.
struct DiagAcc {
  unsigned long long counts[8];
  double sums[8];
  unsigned long long gmax_bits, gscale_bits;
};

constexpr int kDiagBlock = 256;
constexpr int kDiagMaxBlocks = 2048;  // grid-stride: few blocks, so few atomics on the accumulators

// Per-slot diagnostics over a grid-stride loop (at most kDiagMaxBlocks
// blocks): each thread accumulates the counts and sums of its slots, then a
// wavefront reduction and one atomic per block and counter (the accumulators
// share one cache line, whose atomics the memory system takes one at a time).
template <class T, int SER>
__global__ void __launch_bounds__(kDiagBlock)
diag_particles_kernel(Grid g, Tables tab, ParticleArraysT<T> P, double B0, T* __restrict__ Eout,
                      T* __restrict__ Lout, DiagAcc* acc) {
  __shared__ unsigned long long sc[8][kDiagBlock / 64];
  __shared__ double ss[8][kDiagBlock / 64];
  unsigned long long cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P.n; k += stride) {
    const uint8_t t = P.tag[k];
    double E = __builtin_nan(""), L = __builtin_nan("");
    if (t == 0) {
      ++cnt[5];
    } else if (t & kInvalid) {
      ++cnt[6];
    } else {
      const int sp = t & kSpecies;
      if (t & kLeaving) ++cnt[4]; else ++cnt[sp];
      const double u1 = P.u1[k], u2 = P.u2[k], u3 = P.u3[k];
      const double d1 = P.dx1[k], d2 = P.dx2[k];
      if (!(isfinite(u1) && isfinite(u2) && isfinite(u3) && isfinite(d1) && isfinite(d2)))
        ++cnt[6];
      const double x1 = 0.5 * (((double)P.i1p[k] + P.dx1p[k]) + ((double)P.i1[k] + d1));
      const double x2 = 0.5 * (((double)P.i2p[k] + P.dx2p[k]) + ((double)P.i2[k] + d2));
      // r, the clamped sin and cos at the time-centred position, once, for the
      // metric and the Wald potential (the in-cell series of the push on fine
      // grids, the library functions otherwise)
      // (a stale previous position -- the fused pass and the sort do not keep
      // it -- may put the midpoint anywhere: the tables are read only for a
      // midpoint within the grid's cells)
      const double f1 = floor(x1), f2 = floor(x2);
      const bool tabled = f1 >= -1.0 && f1 <= (double)g.n_r && f2 >= 0.0 && f2 <= (double)g.n_th;
      const RSC p = tabled ? rsc_near<SER>(g, tab, (int)f1, x1, (int)f2, x2) : rsc_direct(g, x1, x2);
      const Coeffs m = coeffs_from(g, p);
      const WaldPot w = wald_pot(g, p.r, p.s, p.c, B0);
      const double qm = species_sign(t);
      E = m.alpha * gamma_of(m, u1, u2, u3, mass2_of(t)) - m.beta1 * u1 - qm * w.A0;
      L = u3 + qm * w.A3;
      if (!(t & kLeaving)) {
        sum[sp] += E;
        sum[4 + sp] += L;
      }
    }
    if (Eout) Eout[k] = E;
    if (Lout) Lout[k] = L;
  }
  // wavefront reduction, then one atomic per block and counter
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    for (int off = 32; off > 0; off >>= 1) {
      cnt[q] += __shfl_down(cnt[q], off, 64);
      sum[q] += __shfl_down(sum[q], off, 64);
    }
    if (lane == 0) {
      sc[q][wv] = cnt[q];
      ss[q][wv] = sum[q];
    }
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    const int q = threadIdx.x;
    unsigned long long c = 0;
    double s = 0.0;
    for (int w = 0; w < kDiagBlock / 64; ++w) {
      c += sc[q][w];
      s += ss[q][w];
    }
    if (c) atomicAdd(&acc->counts[q], c);
    if (s != 0.0) atomicAdd(&acc->sums[q], s);
  }
}

// first-order charge sqrt(h) rho = sum q S at the nodes around the current
// positions, two-sided on the axis node rows like the deposited current (the
// particle's mirror image in the nearer axis doubles an axis-row value); the
// lanes of a wavefront that share a cell add their run sum once (every lane
// reaches the run sums: no early return before them)
template <class T>
__global__ void __launch_bounds__(256) charge_kernel(Grid g, ParticleArraysT<T> P, T* __restrict__ Q) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false;
  int i1 = 0, i2 = 0;
  double q = 0.0, w1 = 0.0, w2 = 0.0;
  if (k < P.n) {
    const uint8_t t = P.tag[k];
    const double sg = is_live(t) ? species_sign(t) : 0.0;
    if (sg != 0.0) {
      i1 = P.i1[k];
      i2 = P.i2[k];
      w1 = P.dx1[k];
      w2 = P.dx2[k];
      act = in_deposit_range(g, i1, w1, i2, w2);
      q = sg * g.charge_scale * P.w[k];
    }
  }
  const double e0 = (i2 == 0) ? 2.0 : 1.0, e1 = (i2 + 1 == g.n_th) ? 2.0 : 1.0;
  const T z = (T)0;
  const Runs r = runs_of(act ? (i1 + 2) * g.ld + (i2 + 2) : -1);
  const T s00 = run_sum(act ? (T)(q * (1.0 - w1) * (1.0 - w2) * e0) : z, r);
  const T s01 = run_sum(act ? (T)(q * (1.0 - w1) * w2 * e1) : z, r);
  const T s10 = run_sum(act ? (T)(q * w1 * (1.0 - w2) * e0) : z, r);
  const T s11 = run_sum(act ? (T)(q * w1 * w2 * e1) : z, r);
  if (act && r.head) {
    T* p = Q + ix(g, i1, i2);
    atomic_add(p, s00);
    atomic_add(p + 1, s01);
    atomic_add(p + g.ld, s10);
    atomic_add(p + g.ld + 1, s11);
  }
}

// residual div D - 4 pi rho at nodes i in [n_f + 2, i_hi), j in [0, n_th]:
// the horizon layer overwrites the columns i <= n_f, and from
// i_hi = n_r - max(n_absorb, n_f) on lie the absorbing layer and the columns
// that take filtered charge from particles leaving the grid.  The axis nodes
// take the polar-cap form of Sec. 3.3.2, A_{i+1/2} D^1(i+1/2) - A_{i-1/2}
// D^1(i-1/2) +- sqrt(h) D^2 - 2 pi rho with the two-sided axis-row charge (the
// D^2 flux enters with the opposite orientation at theta = pi).
constexpr int kGaussWaves = 4;  // wavefronts per block of gauss_kernel (256 threads)

template <class T, bool kQ>
__global__ void __launch_bounds__(256) gauss_kernel(Grid g, Tables t, double polar_k, int i_hi, const T* __restrict__ D1,
                             const T* __restrict__ D2, const T* __restrict__ Q,
                             T* __restrict__ res, DiagAcc* acc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y + g.n_filter + 2;
  double rmax = 0.0, smax = 0.0;
  if (j <= g.n_th && i < i_hi) {
    const int64_t o = ix(g, i, j);
    double r;
    if (j >= 1 && j < g.n_th) {
      const double t1 = cell_tab(g, t, i, 1, j, 0).sqrt_h * D1[o];
      const double t2 = cell_tab(g, t, i - 1, 1, j, 0).sqrt_h * D1[o - g.ld];
      const double t3 = cell_tab(g, t, i, 0, j, 1).sqrt_h * D2[o];
      const double t4 = cell_tab(g, t, i, 0, j - 1, 1).sqrt_h * D2[o - 1];
      const double t5 = 4.0 * kPi * Q[o];
      r = (t1 - t2) + (t3 - t4) - t5;
      smax = fmax(fmax(fabs(t1), fabs(t2)), fmax(fmax(fabs(t3), fabs(t4)), fabs(t5)));
    } else {
      auto cap = [&](int ii) {
        const double rr = t.r[1][ii + g.ng];
        const double ra = rr * rr + g.a * g.a;
        return g.dxi * (kQ ? rr - g.r0 : rr) * ra * sqrt(1.0 + 2.0 * g.M * rr / ra) * polar_k;
      };
      const int jd = j == 0 ? 0 : g.n_th - 1;
      const double t1 = cap(i) * D1[o];
      const double t2 = cap(i - 1) * D1[o - g.ld];
      const double t3 = cell_tab(g, t, i, 0, jd, 1).sqrt_h * D2[ix(g, i, jd)];
      const double t5 = 2.0 * kPi * Q[o];
      r = (t1 - t2) + (j == 0 ? t3 : -t3) - t5;
      smax = fmax(fmax(fabs(t1), fabs(t2)), fmax(fabs(t3), fabs(t5)));
    }
    if (res) res[o] = r;
    rmax = fabs(r);
  }
  // wavefront maxima, then the block's (one atomic per block and maximum)
  __shared__ double bm[2][kGaussWaves];
  for (int off = 32; off > 0; off >>= 1) {
    rmax = fmax(rmax, __shfl_down(rmax, off, 64));
    smax = fmax(smax, __shfl_down(smax, off, 64));
  }
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  if (tid % 64 == 0) {
    bm[0][tid / 64] = rmax;
    bm[1][tid / 64] = smax;
  }
  __syncthreads();
  if (tid < 2) {
    double m = bm[tid][0];
    for (int w = 1; w < kGaussWaves; ++w) m = fmax(m, bm[tid][w]);
    atomicMax(tid == 0 ? &acc->gmax_bits : &acc->gscale_bits, (unsigned long long)__double_as_longlong(m));
  }
}

}  // namespace grpic
