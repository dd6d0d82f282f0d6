// inject.hpp -- pair injection where the plasma is strongly magnetised
// (Sec. 4.4 and Sec. 4.5: e+- pairs at temperature T are added wherever the
// magnetisation sigma = B_i B^i / (4 pi n m) reaches a threshold).
//
// Three passes over a cell-sized scratch: the weight of the live e+- of each
// cell (FP64 atomics), the number of pairs each cell injects (0 or n_pairs,
// decided in FP64 from the cell-centred field and the density), an exclusive
// scan of those numbers (the scan kernels of the cell sort), then one thread
// per cell writes its pairs to the slots its scanned offset gives.
#pragma once

#include "init.hpp"
#include "sort.hpp"

namespace grpic {

struct InjectArgs {
  double sigma_th, temp, weight;
  int n_pairs, i_lo, i_hi;
  uint64_t seed;
  uint32_t sub;          // 1 + the call index (0 is the initial loading)
  int64_t first_free;
};

// Sum of the weights of the live, not leaving e+ and e- per cell.
template <class T>
__global__ void __launch_bounds__(256) inject_weights_kernel(Grid g, ParticleArraysT<T> P,
                                                             double* __restrict__ wsum) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P.n) return;
  const uint8_t t = P.tag[k];
  const int s = t & 3;
  if (t == 0 || (t & kLeaving) || (s != 1 && s != 2)) return;
  const int i1 = P.i1[k], i2 = P.i2[k];
  if (i1 < 0 || i1 >= g.n_r || i2 < 0 || i2 >= g.n_th) return;
  atomicAdd(wsum + (int64_t)i1 * g.n_th + i2, (double)P.w[k]);
}

// Pairs injected by each cell: n_pairs where B_i B^i > 0 and
// B_i B^i >= 4 pi sigma_th n, n = kappa (sum w) / sqrt(h), else 0.  B at the
// cell centre: B^1 and B^2 the means of their two faces, B^3 its own value;
// B_i B^i = h_ij B^i B^j with the lower metric there.  Also zeroes the entry
// after the last cell (the scan turns it into the total).
template <class T>
__global__ void __launch_bounds__(256) inject_cells_kernel(Grid g, Tables tab, const T* __restrict__ B1,
                                                           const T* __restrict__ B2,
                                                           const T* __restrict__ B3,
                                                           const double* __restrict__ wsum, InjectArgs a,
                                                           int* __restrict__ count) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ncell = (int64_t)g.n_r * g.n_th;
  if (c > ncell) return;
  if (c == ncell) {
    count[c] = 0;
    return;
  }
  const int i = (int)(c / g.n_th), j = (int)(c % g.n_th);
  int m = 0;
  if (i >= a.i_lo && i < a.i_hi) {
    const Cell e = cell_tab(g, tab, i, 1, j, 1);
    const int64_t o = ix(g, i, j);
    const double b1 = 0.5 * ((double)B1[o] + (double)B1[o + g.ld]);
    const double b2 = 0.5 * ((double)B2[o] + (double)B2[o + 1]);
    const double b3 = (double)B3[o];
    const double bb = e.hl11 * b1 * b1 + 2.0 * e.hl13 * b1 * b3 + e.hl22 * b2 * b2 + e.hl33 * b3 * b3;
    const double n = g.charge_scale * wsum[c] / e.sqrt_h;
    if (bb > 0.0 && bb >= 4.0 * kPi * a.sigma_th * n) m = a.n_pairs;
  }
  count[c] = m;
}

// One thread per cell: pair k = off[c] + e (e < the cell's count) goes to
// slots first_free + 2k (e+) and first_free + 2k + 1 (e-) at one position,
// offsets uniform in the cell (Philox stream 0 of pair k), momenta isotropic
// Maxwell-Juttner at temp in the FIDO tetrad frame there (streams 1, 2 of
// particle 2k + s); pairs past the last slot are not written.
template <class T>
__global__ void __launch_bounds__(256) inject_pairs_kernel(Grid g, ParticleArraysT<T> P,
                                                           const int* __restrict__ off, InjectArgs a) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ncell = (int64_t)g.n_r * g.n_th;
  if (c >= ncell) return;
  const int64_t k0 = off[c], m = (int64_t)off[c + 1] - k0;
  const int i = (int)(c / g.n_th), j = (int)(c % g.n_th);
  for (int64_t e = 0; e < m; ++e) {
    const int64_t k = k0 + e;
    const int64_t q0 = a.first_free + 2 * k;
    if (q0 + 1 >= P.n) return;
    uint32_t w[4];
    draw4(a.seed, (uint32_t)k, 0u, 0u, w, a.sub);
    const double dx1 = u_low(w[0]), dx2 = u_low(w[1]);
    const Tetrad tf = tetrad_at(g, (double)i + dx1, (double)j + dx2);
    for (int s = 0; s < 2; ++s) {
      double uh[3], u1, u2, u3;
      maxwell_juttner(a.seed, (uint32_t)(2 * k + s), a.temp, uh, a.sub);
      hat_to_cov(tf, uh, u1, u2, u3);
      store_particle(P, q0 + s, i, j, dx1, dx2, u1, u2, u3, (uint8_t)(s == 0 ? 1 : 2), a.weight);
    }
  }
}

}  // namespace grpic
