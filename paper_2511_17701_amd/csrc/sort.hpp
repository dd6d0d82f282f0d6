// sort.hpp -- counting sort of the particle slots by cell (c = i1 * n_th + i2).
//
// Not part of the paper's method: a layout device that keeps particles of one
// cell adjacent in memory, so that a wavefront streams contiguous SoA data,
// gathers from a few neighbouring field entries, and the deposit's per-block
// footprint stays inside its shared-memory tile.  Empty and leaving slots get
// the key n_cells and end up (emptied) after all live particles.
#pragma once

#include "particles.hpp"

namespace grpic {

constexpr int kScanBlock = 1024;  // elements scanned per block (4 per thread)

template <class T>
__device__ inline int sort_key(const Grid& g, const ParticleArraysT<T>& P, int64_t k) {
  const uint8_t t = P.tag[k];
  const int ncell = g.n_r * g.n_th;
  if (!is_live(t) || (t & kLeaving)) return ncell;
  const int i1 = P.i1[k], i2 = P.i2[k];
  if (i1 < 0 || i1 >= g.n_r || i2 < 0 || i2 >= g.n_th) return ncell;
  return i1 * g.n_th + i2;
}

// Runs of equal keys in consecutive lanes of a wavefront (particles arrive
// nearly sorted, so a wave holds a few runs): one atomic per run.
struct Run {
  int key, head, len;  // this lane's key, its run's first lane, the run length
  bool first;          // lane is the first of its run
};

__device__ inline Run wave_run(int key) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  const bool first = lane == 0 || prev != key;
  const unsigned long long heads = __ballot(first);
  const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1);
  Run r;
  r.key = key;
  r.first = first;
  r.head = 63 - __clzll(heads & upto);
  const unsigned long long after = lane == 63 ? 0ull : (heads >> (lane + 1));
  r.len = first ? (after ? __ffsll((long long)after) : 64 - lane) : 0;
  return r;
}

// Each wavefront of the rank pass takes kSortPer consecutive chunks of 64
// slots (one slot per lane in each), so that one round trip of its counter
// atomics covers kSortPer chunks.
constexpr int kSortPer = 8;

__device__ inline int64_t sort_first_slot() {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  return wave * 64 * kSortPer + (threadIdx.x & 63);
}

// Counts the slots of each key and gives every slot its rank among the slots
// of its key: the first lane of each run claims the run's ranks with one
// returning atomic on the key's counter (all of a wavefront's kSortPer
// claims are in flight before the first is waited for), the other lanes of
// the run follow it.  The rank is written to the source's i1p (the previous
// position is scratch between a push and its deposit, and the sort does not
// carry it), so the scatter needs no atomics.
template <class T>
__global__ void __launch_bounds__(256) sort_rank_kernel(Grid g, ParticleArraysT<T> P, int* __restrict__ counts) {
  const int64_t k0 = sort_first_slot();
  int key[kSortPer], base[kSortPer];
  Run r[kSortPer];
#pragma unroll
  for (int c = 0; c < kSortPer; ++c) {
    const int64_t k = k0 + 64 * c;
    key[c] = k < P.n ? sort_key(g, P, k) : -1;  // -1: past the end (own run)
  }
#pragma unroll
  for (int c = 0; c < kSortPer; ++c) {
    r[c] = wave_run(key[c]);
    base[c] = 0;
    if (r[c].first && key[c] >= 0) base[c] = atomicAdd(counts + key[c], r[c].len);
  }
#pragma unroll
  for (int c = 0; c < kSortPer; ++c) {
    const int b = __shfl(base[c], r[c].head, 64);
    const int64_t k = k0 + 64 * c;
    if (key[c] >= 0) P.i1p[k] = b + ((threadIdx.x & 63) - r[c].head);
  }
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

// Moves slot k of S to slot off[key] + rank of D (rank from sort_rank_kernel,
// in S.i1p; off the exclusive scan of the key counts); emptied slots get tag
// 0.  No atomics: every load and store of a wavefront is independent, so the
// pass streams at the memory system's rate.  The previous position (scratch
// between a push and its deposit) is not carried.
template <class T>
__global__ void __launch_bounds__(256) sort_scatter_kernel(Grid g, ParticleArraysT<T> S, ParticleArraysT<T> D,
                                                           const int* __restrict__ off) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= S.n) return;
  const int ncell = g.n_r * g.n_th;
  const int key = sort_key(g, S, k);
  const int64_t o = (int64_t)off[key] + S.i1p[k];
  if (key == ncell) {
    D.tag[o] = 0;
    return;
  }
  D.i1[o] = S.i1[k];
  D.i2[o] = S.i2[k];
  D.dx1[o] = S.dx1[k];
  D.dx2[o] = S.dx2[k];
  D.u1[o] = S.u1[k];
  D.u2[o] = S.u2[k];
  D.u3[o] = S.u3[k];
  D.w[o] = S.w[k];
  D.phi[o] = S.phi[k];
  D.tag[o] = S.tag[k];
}

}  // namespace grpic
