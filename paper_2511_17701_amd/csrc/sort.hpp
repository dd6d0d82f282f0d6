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

// Each wavefront takes kSortPer consecutive chunks of 64 slots (one slot per
// lane in each), so that one round trip of its cell-offset atomics covers
// kSortPer chunks.
constexpr int kSortPer = 4;

__device__ inline int64_t sort_first_slot() {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  return wave * 64 * kSortPer + (threadIdx.x & 63);
}

template <class T>
__global__ void __launch_bounds__(256) sort_count_kernel(Grid g, ParticleArraysT<T> P,
                                                         int* __restrict__ counts) {
  const int64_t k0 = sort_first_slot();
#pragma unroll
  for (int c = 0; c < kSortPer; ++c) {
    const int64_t k = k0 + 64 * c;
    const int key = k < P.n ? sort_key(g, P, k) : -1;  // -1: past the end (own run)
    const Run r = wave_run(key);
    if (r.first && key >= 0) atomicAdd(counts + key, r.len);
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

// Moves slot k of S to its cell's next free slots in D; emptied slots get tag
// 0.  The previous position (scratch between a push and its deposit) is not
// carried.  A run of equal keys in a chunk takes consecutive slots in lane
// order; the order of runs of one cell follows the order of the atomics.  All
// of a wavefront's slots are read, and all its offsets claimed, before the
// first offset is waited for.
template <class T>
struct SlotT {
  int i1, i2;
  T dx1, dx2, u1, u2, u3, w, phi;
  uint8_t tag;
};

template <class T>
__global__ void __launch_bounds__(256) sort_scatter_kernel(Grid g, ParticleArraysT<T> S, ParticleArraysT<T> D,
                                                           int* __restrict__ off) {
  const int64_t k0 = sort_first_slot();
  const int ncell = g.n_r * g.n_th;
  int key[kSortPer];
  SlotT<T> v[kSortPer];
#pragma unroll
  for (int c = 0; c < kSortPer; ++c) {
    const int64_t k = k0 + 64 * c;
    key[c] = k < S.n ? sort_key(g, S, k) : -1;
    v[c] = SlotT<T>{};
    if (key[c] >= 0 && key[c] < ncell) {
      v[c].i1 = S.i1[k];
      v[c].i2 = S.i2[k];
      v[c].dx1 = S.dx1[k];
      v[c].dx2 = S.dx2[k];
      v[c].u1 = S.u1[k];
      v[c].u2 = S.u2[k];
      v[c].u3 = S.u3[k];
      v[c].w = S.w[k];
      v[c].phi = S.phi[k];
      v[c].tag = S.tag[k];
    }
  }
  Run r[kSortPer];
  int base[kSortPer];
#pragma unroll
  for (int c = 0; c < kSortPer; ++c) {
    r[c] = wave_run(key[c]);
    base[c] = 0;
    if (r[c].first && key[c] >= 0) base[c] = atomicAdd(off + key[c], r[c].len);
  }
#pragma unroll
  for (int c = 0; c < kSortPer; ++c) {
    const int b = __shfl(base[c], r[c].head, 64);
    if (key[c] < 0) continue;
    const int64_t o = (int64_t)b + ((threadIdx.x & 63) - r[c].head);
    if (key[c] == ncell) {
      D.tag[o] = 0;
      continue;
    }
    D.i1[o] = v[c].i1;
    D.i2[o] = v[c].i2;
    D.dx1[o] = v[c].dx1;
    D.dx2[o] = v[c].dx2;
    D.u1[o] = v[c].u1;
    D.u2[o] = v[c].u2;
    D.u3[o] = v[c].u3;
    D.w[o] = v[c].w;
    D.phi[o] = v[c].phi;
    D.tag[o] = v[c].tag;
  }
}

}  // namespace grpic
