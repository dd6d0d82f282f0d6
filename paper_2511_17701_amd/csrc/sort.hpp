// sort.hpp -- counting sort of the particle slots by cell (c = i1 * n_th + i2).
//
// Not part of the paper's method: a layout device that keeps particles of one
// cell adjacent in memory, so that a wavefront streams contiguous SoA data,
// gathers from a few neighbouring field entries, and the deposit's per-block
// footprint stays inside its shared-memory tile.  Empty and leaving slots get
// the key n_cells: they take no counter and no rank and are not moved; the
// destination's slots after the live particles get tag 0.
#pragma once

#include "particles.hpp"

namespace grpic {

constexpr int kScanBlock = 1024;  // elements scanned per block (4 per thread)

template <class T>
__device__ inline int sort_key(const Grid& g, const ParticleArraysT<T>& P, int64_t k) {
  const uint8_t t = P.tag[k];
  if (!is_live(t) || (t & kLeaving)) return g.n_r * g.n_th;
  return cell_key(g, t, P.i1[k], P.i2[k]);
}

// The rank pass takes kRankBlock consecutive slots per block of 256 threads
// (8 per thread) and counts them in a RankTable of kRankTable cells.
constexpr int kRankBits = 12;
constexpr int kRankBlock = 2048, kRankTable = 1 << kRankBits;
static_assert(kRankTable >= 2 * kRankBlock, "rank table too small for a block");

// Counts the live slots of each cell and gives every live slot its rank among
// the slots of its cell (block counting in an LDS hash table, one claim per
// cell and block: RankTable).  Ten steps after a sort, neighbouring slots
// mostly hold particles of different (nearby) cells, so runs of equal cells
// are short (about 2 slots at 16 particles per cell), while a block's slots
// fall in a few hundred distinct cells (measured: 262 of 2048 on a 4096^2
// grid at 16 particles per cell, 83 on 2048^2 at 90).  The rank is written to
// the source's i1p (the previous position is scratch between a push and its
// deposit, and the sort does not carry it), so the scatter needs no atomics.
// The fused push + deposit pass can do the same per block of its own
// (rank_fused), which makes this pass unnecessary.
template <class T>
__global__ void __launch_bounds__(256) sort_rank_kernel(Grid g, ParticleArraysT<T> P, int* __restrict__ counts) {
  RankTable<kRankBits>& rt = block_rank_table<kRankBits>();
  const int ncell = g.n_r * g.n_th;
  const int64_t k0 = (int64_t)blockIdx.x * kRankBlock;
  const int t = threadIdx.x;
  rank_clear(rt);
  __syncthreads();
  constexpr int kQ = kRankBlock / 256;
  int entry[kQ], local[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int64_t k = k0 + q * 256 + t;  // consecutive threads on consecutive slots
    const int key = k < P.n ? sort_key(g, P, k) : ncell;
    entry[q] = key < ncell ? rank_insert(rt, key, local[q]) : -1;
  }
  __syncthreads();
  rank_claim<kRankBits, 256>(rt, counts);
#pragma unroll
  for (int q = 0; q < kQ; ++q)
    if (entry[q] >= 0) P.i1p[k0 + q * 256 + t] = rt.n[entry[q]] + local[q];
}

// Exclusive scan of n ints in place, three phases: per-block scan (block sums
// out), scan of the block sums (one block), add the scanned block sums.
__device__ inline int block_exclusive_scan(int v, int* sh) {
  // Hillis-Steele over 256 threads in LDS
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(256) scan_blocks_kernel(int* __restrict__ a, int64_t n,
                                                          int* __restrict__ sums) {
  __shared__ int sh[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
  int v[4];
  int tot = 0;
  for (int q = 0; q < 4; ++q) {
    v[q] = base + q < n ? a[base + q] : 0;
    tot += v[q];
  }
  const int ex = block_exclusive_scan(tot, sh);
  int run = ex;
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) a[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == 255) sums[blockIdx.x] = ex + tot;
}

__global__ void __launch_bounds__(256) scan_sums_kernel(int* __restrict__ sums, int nb) {
  __shared__ int sh[256];
  // serial over chunks of 256 (nb is small: n / 1024)
  int carry = 0;
  for (int base = 0; base < nb; base += 256) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? sums[i] : 0;
    const int ex = block_exclusive_scan(v, sh);
    if (i < nb) sums[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 255) sh[0] = ex + v;
    __syncthreads();
    carry += sh[0];
    __syncthreads();
  }
}

__global__ void scan_add_kernel(int* __restrict__ a, int64_t n, const int* __restrict__ sums) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += sums[i / kScanBlock];
}

// Source loads of the scatter: non-temporal in the single-precision form,
// which leaves the L2 to the destination lines that the wavefronts fill in
// pieces (measured at 4096^2, 16 particles per cell: -3 % for a sort after 10
// steps of motion, -18 % for a re-sort); plain in double precision, where the
// same loads gained nothing (4096^2 at 16 and 2048^2 at 90 particles per
// cell: the same or up to 5 % slower, against a spread of several per cent
// between single sorts).
template <class T, class V>
__device__ inline V scatter_load(const V* p) {
  if constexpr (sizeof(T) == 4) return __builtin_nontemporal_load(p);
  else return *p;
}

// Moves live slot k of S to slot off[key] + rank of D (rank from
// sort_rank_kernel, in S.i1p; off the exclusive scan of the cell counts).  No
// atomics: every load and store of a wavefront is independent, so the pass
// streams at the memory system's rate.  Empty and leaving slots are not
// moved (sort_clear_tail_kernel empties the destination after the live
// slots).  The previous position (scratch between a push and its deposit) is
// not carried.
template <class T>
__global__ void __launch_bounds__(256) sort_scatter_kernel(Grid g, ParticleArraysT<T> S, ParticleArraysT<T> D,
                                                           const int* __restrict__ off) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= S.n) return;
  const uint8_t t = scatter_load<T>(S.tag + k);
  const int i1 = scatter_load<T>(S.i1 + k), i2 = scatter_load<T>(S.i2 + k);
  const int key = cell_key(g, t, i1, i2);
  if (key == g.n_r * g.n_th) return;
  const int64_t o = (int64_t)off[key] + scatter_load<T>(S.i1p + k);
  if (o < 0 || o >= D.n) return;  // ranks that do not belong to these counts (a caller's error)
  D.i1[o] = i1;
  D.i2[o] = i2;
  D.dx1[o] = scatter_load<T>(S.dx1 + k);
  D.dx2[o] = scatter_load<T>(S.dx2 + k);
  D.u1[o] = scatter_load<T>(S.u1 + k);
  D.u2[o] = scatter_load<T>(S.u2 + k);
  D.u3[o] = scatter_load<T>(S.u3 + k);
  D.w[o] = scatter_load<T>(S.w + k);
  D.phi[o] = scatter_load<T>(S.phi + k);
  D.tag[o] = t;
}

// Tag 0 on the destination slots from the live count (*live, the scan's
// total) to n: a grid-stride loop, so the launch can be small.
__global__ void __launch_bounds__(256) sort_clear_tail_kernel(uint8_t* __restrict__ tag, int64_t n,
                                                              const int* __restrict__ live) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)*live + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) tag[k] = 0;
}

}  // namespace grpic
