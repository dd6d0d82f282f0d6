// grpic.hip -- C ABI of libgrpic.so (declared in include/grpic.h): argument
// checks, per-context tables, and the launch sequences of the PIC-loop stages.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "grpic.h"
#include "adjoint.hpp"
#include "diag.hpp"
#include "inject.hpp"
#include "sort.hpp"

using namespace grpic;

struct grpic_ctx {
  grpic_params prm;
  Grid g;
  int device;
  bool f32;        // single-precision storage (GRPIC_FP32)
  double* tables;  // r[2], s[2], c[2] (n + 2 ng each), then float r, sin, cos at nodes
  Tables tab;
  DiagAcc* acc;    // device accumulators for diagnostics
  double polar_k;  // 1 - cos(theta(x2 = 1/2)): the polar cap of the axis update
  int* sort_off;   // n_cells + 1 counts / offsets, then block sums, then n_live
  int* sort_sums;
  int* sort_live;
  double* inj_w;   // per-cell e+- weight of the pair injection (allocated on first use)
  int* static_scratch;  // this device's address of `scratch` (grpic_sort_noalloc)
  // grpic_push_deposit_ranked: the sort scratch its rank pass fills
  // (allocated on first use) and the particle set it ranked, which the next
  // grpic_sort_ranked must be given
  int* rank_off;
  bool ranked;
  const void* ranked_i1p;
  int64_t ranked_n;
};

// Scratch of grpic_sort_noalloc, which allocates nothing: the cell counters /
// offsets of grids of up to kStaticSortCells cells, the scan's block sums and
// the live count (kStaticSortInts ints, 64.1 MiB).  Every GPU the library runs
// on holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress gives on that device.
constexpr int64_t kStaticSortCells = (int64_t)1 << 24;  // 4096 x 4096
constexpr int64_t kStaticSortKeys = kStaticSortCells + 1;
constexpr int64_t kStaticSortInts = kStaticSortKeys + (kStaticSortKeys + grpic::kScanBlock - 1) / grpic::kScanBlock + 1;
static __device__ __align__(256) int scratch[kStaticSortInts];

namespace grpic {
__global__ void fill_int_kernel(int64_t n, int* __restrict__ p, int v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}
__global__ void copy_int_kernel(const int* __restrict__ src, int* __restrict__ dst) { *dst = *src; }
}  // namespace grpic

namespace {

thread_local std::string g_err;

grpic_status fail(grpic_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
grpic_status fail(grpic_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(GRPIC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_CHECK(name)                                                                  \
  do {                                                                                      \
    hipError_t e_ = hipGetLastError();                                                      \
    if (e_ != hipSuccess) return fail(GRPIC_EHIP, "launch %s: %s", name, hipGetErrorString(e_)); \
  } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

grpic_status check_ctx(const grpic_ctx* c) {
  if (!c) return fail(GRPIC_EINVAL, "null context");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != c->device) return fail(GRPIC_ESTATE, "context made on device %d, current is %d", c->device, dev);
  return GRPIC_OK;
}

grpic_status check_fields(const grpic_ctx* c, const grpic_fields* F) {
  if (!F) return fail(GRPIC_EINVAL, "null field set");
  void* const* p = &F->D[0];
  const int n = c->f32 ? 39 : 33;  // the compensation planes Dc, Bc in the FP32 form
  for (int k = 0; k < n; ++k)
    if (!p[k]) return fail(GRPIC_EINVAL, "field plane %d is null", k);
  return GRPIC_OK;
}

grpic_status check_particles(const grpic_particles* P) {
  if (!P) return fail(GRPIC_EINVAL, "null particle set");
  if (P->n < 0) return fail(GRPIC_EINVAL, "negative particle count");
  if (P->n == 0) return GRPIC_OK;
  if (!P->i1 || !P->i2 || !P->dx1 || !P->dx2 || !P->u1 || !P->u2 || !P->u3 || !P->w || !P->phi ||
      !P->i1p || !P->i2p || !P->dx1p || !P->dx2p || !P->tag)
    return fail(GRPIC_EINVAL, "particle array pointer is null");
  return GRPIC_OK;
}

template <class T>
ParticleArraysT<T> arrays(const grpic_particles* P) {
  ParticleArraysT<T> a;
  a.i1 = P->i1;
  a.i2 = P->i2;
  a.dx1 = (T*)P->dx1;
  a.dx2 = (T*)P->dx2;
  a.u1 = (T*)P->u1;
  a.u2 = (T*)P->u2;
  a.u3 = (T*)P->u3;
  a.w = (T*)P->w;
  a.phi = (T*)P->phi;
  a.i1p = P->i1p;
  a.i2p = P->i2p;
  a.dx1p = (T*)P->dx1p;
  a.dx2p = (T*)P->dx2p;
  a.tag = P->tag;
  a.n = P->n;
  return a;
}

template <class T>
TriT<T> tri(void* const p[3]) {
  return TriT<T>{{(T*)p[0], (T*)p[1], (T*)p[2]}};
}
template <class T>
CTriT<T> ctri(void* const p[3]) {
  return CTriT<T>{{(const T*)p[0], (const T*)p[1], (const T*)p[2]}};
}
// compensation planes of an evolved triple (single-precision form only)
template <class T>
TriT<T> comp(const grpic_ctx* c, void* const p[3]) {
  return c->f32 ? tri<T>(p) : TriT<T>{{nullptr, nullptr, nullptr}};
}
template <class T>
TriT<T> none() {
  return TriT<T>{{nullptr, nullptr, nullptr}};
}

constexpr int kB = 256;
inline unsigned blocks(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

// 2-D launch over an (ni x nj) range, threads along j: blocks of 2 rows of
// 128 (measured against 64 x 4, 256 x 1 and 64 x 8 on the field stages: the
// fastest at 4096^2, within 1 % at 2048^2 and 512^2)
inline dim3 grid2(int ni, int nj) { return dim3((nj + 127) / 128, (ni + 1) / 2); }
const dim3 kBlock2(128, 2);

const int3 kStagD1 = {1, 0, 0}, kStagD2 = {0, 1, 0};  // x1 / x2 staggering of D^i, J^i
const int3 kStagB1 = {0, 1, 1}, kStagB2 = {1, 0, 1};  // x1 / x2 staggering of B^i

// boundaries of an updated triple: horizon layer + absorbing layer (radial =
// 1), then the axis
template <class T>
grpic_status field_bc(grpic_ctx* c, TriT<T> X, TriT<T> L, CTriT<T> X0, bool is_B, hipStream_t s,
                      int radial = 1) {
  const Grid& g = c->g;
  const BcRows rows = bc_rows(g);
  if (radial && rows.n_hor + rows.n_abs > 0) {
    const dim3 grid((unsigned)((g.ld + kB - 1) / kB), (unsigned)(rows.n_hor + rows.n_abs));
    hipLaunchKernelGGL(bc_radial_kernel<T>, grid, dim3(kB), 0, s, g, X, L, X0, is_B ? kStagB1 : kStagD1);
    LAUNCH_CHECK("bc_radial");
  }
  const int rpb = bc_axis_rows(g, kB);
  hipLaunchKernelGGL(bc_axis_kernel<T>, dim3((unsigned)((g.n_r + 2 * g.ng + rpb - 1) / rpb)), dim3(kB), 0, s, g, X,
                     L, is_B ? kStagB2 : kStagD2, is_B ? 1 : 2);
  LAUNCH_CHECK("bc_axis");
  return GRPIC_OK;
}

// n_f binomial passes (Sec. 3.3.4) over the ncomp planes of A, up to
// kFMaxPasses per launch of the register-strip kernel, alternating between A
// and B; *out is the triple that holds the result (A when n_f = 0).
constexpr int kFStripRows = 32;  // output rows per wavefront (48 and 64: within 3 % at 4096^2)

template <class T, int P>
void launch_filter_strips(const Grid& g, int ncomp, TriT<T> dst, CTriT<T> src, int3 half2, int3 parity,
                          hipStream_t s) {
  constexpr int kSR = kFStripRows;
  const int nrow = g.n_r + 2 * g.ng;
  const bool small = nrow < kSR + 2 * P;  // fewer plane rows than a strip stages
  const int strips = small ? filter_strips_r<P, kSR, true>(nrow) : filter_strips_r<P, kSR, false>(nrow);
  const dim3 grid((unsigned)filter_strips_theta((int)g.ld), (unsigned)((strips + 3) / 4), (unsigned)ncomp);
  if (small)
    hipLaunchKernelGGL((filter_strip_kernel<T, P, kSR, true>), grid, dim3(256), 0, s, g, dst, src, half2, parity);
  else
    hipLaunchKernelGGL((filter_strip_kernel<T, P, kSR, false>), grid, dim3(256), 0, s, g, dst, src, half2, parity);
}

template <class T>
grpic_status filter_passes(grpic_ctx* c, TriT<T> A, TriT<T> B, int ncomp, int3 half2, int3 parity, hipStream_t s,
                           TriT<T>* out) {
  const Grid& g = c->g;
  bool in_A = true;  // where the latest result is
  for (int done = 0; done < g.n_filter;) {
    // at most kFMaxPasses per launch, and a single-pass launch only for n_f = 1
    // (5 passes as 3 + 2: the single-pass kernel needs the most registers)
    int passes = std::min(kFMaxPasses, g.n_filter - done);
    if (g.n_filter - done - passes == 1) passes -= 1;
    const TriT<T>& dst = in_A ? B : A;
    const TriT<T>& src = in_A ? A : B;
    CTriT<T> srcc{{src.p[0], src.p[1], src.p[2]}};
    switch (passes) {
      case 1: launch_filter_strips<T, 1>(g, ncomp, dst, srcc, half2, parity, s); break;
      case 2: launch_filter_strips<T, 2>(g, ncomp, dst, srcc, half2, parity, s); break;
      case 3: launch_filter_strips<T, 3>(g, ncomp, dst, srcc, half2, parity, s); break;
      default: launch_filter_strips<T, 4>(g, ncomp, dst, srcc, half2, parity, s); break;
    }
    LAUNCH_CHECK("filter_strip");
    done += passes;
    in_A = !in_A;
  }
  const TriT<T>& res = in_A ? A : B;
  for (int k = 0; k < 3; ++k) out->p[k] = res.p[k];
  return GRPIC_OK;
}

// ------------------------------------------------------------------ stages by storage type

template <class T>
grpic_status particles_init_impl(grpic_ctx* c, const grpic_particles* P, int64_t n_pairs, int32_t ppc,
                                 double T_, int64_t n_geo, uint64_t seed, hipStream_t s) {
  const Grid& g = c->g;
  const ParticleArraysT<T> a = arrays<T>(P);
  if (n_pairs > 0) {
    hipLaunchKernelGGL(load_pairs_kernel<T>, dim3(blocks(n_pairs)), dim3(kB), 0, s, g, a, n_pairs, ppc, T_,
                       seed);
    LAUNCH_CHECK("load_pairs");
  }
  if (n_geo > 0) {
    hipLaunchKernelGGL(load_geodesics_kernel<T>, dim3(blocks(n_geo)), dim3(kB), 0, s, g, a, 2 * n_pairs,
                       n_geo, seed);
    LAUNCH_CHECK("load_geodesics");
  }
  return GRPIC_OK;
}

template <class T>
grpic_status wald_impl(grpic_ctx* c, const grpic_fields* F, double B0, hipStream_t s) {
  const Grid& g = c->g;
  void* const* pl = &F->D[0];
  for (int k = 0; k < (c->f32 ? 39 : 33); ++k) {
    hipLaunchKernelGGL(fill_kernel<T>, dim3(blocks(g.plane)), dim3(kB), 0, s, g.plane, (T*)pl[k], 0.0);
    LAUNCH_CHECK("fill");
  }
  hipLaunchKernelGGL(wald_kernel<T>, grid2(g.n_r + 2 * g.ng, g.n_th + 2 * g.ng), kBlock2, 0, s, g, c->tab,
                     tri<T>(F->D), tri<T>(F->B), B0);
  LAUNCH_CHECK("wald");
  grpic_status st;
  if ((st = field_bc<T>(c, tri<T>(F->D), none<T>(), ctri<T>(F->Dinit), false, s, 0))) return st;
  if ((st = field_bc<T>(c, tri<T>(F->B), none<T>(), ctri<T>(F->Binit), true, s, 0))) return st;
  void* const* dst[4] = {F->D0, F->B0, F->Dinit, F->Binit};
  void* const* src[4] = {F->D, F->B, F->D, F->B};
  for (int k = 0; k < 4; ++k) {
    hipLaunchKernelGGL(copy_kernel<T>, dim3(blocks(g.plane)), dim3(kB), 0, s, g.plane, tri<T>(dst[k]),
                       ctri<T>(src[k]));
    LAUNCH_CHECK("copy");
  }
  return GRPIC_OK;
}

template <class T>
grpic_status monopole_impl(grpic_ctx* c, const grpic_fields* F, double B0, hipStream_t s) {
  const Grid& g = c->g;
  void* const* pl = &F->D[0];
  for (int k = 0; k < (c->f32 ? 39 : 33); ++k) {
    hipLaunchKernelGGL(fill_kernel<T>, dim3(blocks(g.plane)), dim3(kB), 0, s, g.plane, (T*)pl[k], 0.0);
    LAUNCH_CHECK("fill");
  }
  hipLaunchKernelGGL(monopole_kernel<T>, grid2(g.n_r + 2 * g.ng, g.n_th + 2 * g.ng), kBlock2, 0, s, g, c->tab,
                     (T*)F->B[0], B0);
  LAUNCH_CHECK("monopole");
  grpic_status st;
  if ((st = field_bc<T>(c, tri<T>(F->D), none<T>(), ctri<T>(F->Dinit), false, s, 0))) return st;
  if ((st = field_bc<T>(c, tri<T>(F->B), none<T>(), ctri<T>(F->Binit), true, s, 0))) return st;
  void* const* dst[4] = {F->D0, F->B0, F->Dinit, F->Binit};
  void* const* src[4] = {F->D, F->B, F->D, F->B};
  for (int k = 0; k < 4; ++k) {
    hipLaunchKernelGGL(copy_kernel<T>, dim3(blocks(g.plane)), dim3(kB), 0, s, g.plane, tri<T>(dst[k]),
                       ctri<T>(src[k]));
    LAUNCH_CHECK("copy");
  }
  return GRPIC_OK;
}

grpic_status push_impl(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P, hipStream_t s) {
  const dim3 grid(blocks(P->n));
  if (c->f32) {
    GatherPlanesT<float> gp;
    for (int k = 0; k < 3; ++k) {
      gp.D[k] = (const float*)F->D[k];
      gp.B[k] = (const float*)F->B0[k];
    }
    switch (c->g.ser) {
      case 2: hipLaunchKernelGGL((push_kernel_f32<2>), grid, dim3(kB), 0, s, c->g, c->tab, gp, arrays<float>(P)); break;
      case 1: hipLaunchKernelGGL((push_kernel_f32<1>), grid, dim3(kB), 0, s, c->g, c->tab, gp, arrays<float>(P)); break;
      default: hipLaunchKernelGGL((push_kernel_f32<0>), grid, dim3(kB), 0, s, c->g, c->tab, gp, arrays<float>(P)); break;
    }
  } else {
    GatherPlanesT<double> gp;
    for (int k = 0; k < 3; ++k) {
      gp.D[k] = (const double*)F->D[k];
      gp.B[k] = (const double*)F->B0[k];
    }
    switch (c->g.ser) {
      case 2: hipLaunchKernelGGL((push_kernel<2>), grid, dim3(kB), 0, s, c->g, c->tab, gp, arrays<double>(P)); break;
      case 1: hipLaunchKernelGGL((push_kernel<1>), grid, dim3(kB), 0, s, c->g, c->tab, gp, arrays<double>(P)); break;
      default: hipLaunchKernelGGL((push_kernel<0>), grid, dim3(kB), 0, s, c->g, c->tab, gp, arrays<double>(P)); break;
    }
  }
  LAUNCH_CHECK("push");
  return GRPIC_OK;
}

// counts: null, or the sort's zeroed cell counters, which the ranked kernels
// fill (with each live slot's rank in its cell written to i1p)
template <bool kRank>
void launch_push_deposit(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P, int* counts,
                         hipStream_t s) {
  if (c->f32) {
    constexpr int kBk = dep_block<float>();
    const dim3 grid((unsigned)((P->n + kBk - 1) / kBk));
    GatherPlanesT<float> gp;
    for (int k = 0; k < 3; ++k) {
      gp.D[k] = (const float*)F->D[k];
      gp.B[k] = (const float*)F->B0[k];
    }
    CurrentPlanesT<float> cp{{(float*)F->J[0], (float*)F->J[1], (float*)F->J[2]}};
    const ParticleArraysT<float> a = arrays<float>(P);
    switch (c->g.ser) {
      case 2: hipLaunchKernelGGL((push_deposit_kernel_f32<2, kRank>), grid, dim3(kBk), 0, s, c->g, c->tab, gp, a, cp, counts); break;
      case 1: hipLaunchKernelGGL((push_deposit_kernel_f32<1, kRank>), grid, dim3(kBk), 0, s, c->g, c->tab, gp, a, cp, counts); break;
      default: hipLaunchKernelGGL((push_deposit_kernel_f32_lib<kRank>), grid, dim3(kBk), 0, s, c->g, c->tab, gp, a, cp, counts); break;
    }
  } else {
    constexpr int kBk = dep_block<double>();
    const dim3 grid((unsigned)((P->n + kBk - 1) / kBk));
    GatherPlanesT<double> gp;
    for (int k = 0; k < 3; ++k) {
      gp.D[k] = (const double*)F->D[k];
      gp.B[k] = (const double*)F->B0[k];
    }
    CurrentPlanesT<double> cp{{(double*)F->J[0], (double*)F->J[1], (double*)F->J[2]}};
    const ParticleArraysT<double> a = arrays<double>(P);
    switch (c->g.ser) {
      case 2: hipLaunchKernelGGL((push_deposit_kernel<2, kRank>), grid, dim3(kBk), 0, s, c->g, c->tab, gp, a, cp, counts); break;
      case 1: hipLaunchKernelGGL((push_deposit_kernel<1, kRank>), grid, dim3(kBk), 0, s, c->g, c->tab, gp, a, cp, counts); break;
      default: hipLaunchKernelGGL((push_deposit_kernel_lib<kRank>), grid, dim3(kBk), 0, s, c->g, c->tab, gp, a, cp, counts); break;
    }
  }
}

grpic_status push_deposit_impl(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P, int* counts,
                               hipStream_t s) {
  if (counts) launch_push_deposit<true>(c, F, P, counts, s);
  else launch_push_deposit<false>(c, F, P, nullptr, s);
  LAUNCH_CHECK("push_deposit");
  return GRPIC_OK;
}

template <class T>
grpic_status deposit_impl(grpic_ctx* c, const grpic_particles* P, const grpic_fields* F, hipStream_t s) {
  CurrentPlanesT<T> cp{{(T*)F->J[0], (T*)F->J[1], (T*)F->J[2]}};
  constexpr int kBk = dep_block<T>();
  const dim3 grid((unsigned)((P->n + kBk - 1) / kBk));
  switch (c->g.ser) {
    case 2: hipLaunchKernelGGL((deposit_kernel<T, 2>), grid, dim3(kBk), 0, s, c->g, c->tab, arrays<T>(P), cp); break;
    case 1: hipLaunchKernelGGL((deposit_kernel<T, 1>), grid, dim3(kBk), 0, s, c->g, c->tab, arrays<T>(P), cp); break;
    default: hipLaunchKernelGGL((deposit_kernel<T, 0>), grid, dim3(kBk), 0, s, c->g, c->tab, arrays<T>(P), cp); break;
  }
  LAUNCH_CHECK("deposit");
  return GRPIC_OK;
}

// Device scratch of one sort: n_cells + 1 counters / offsets, the scan's
// block sums, the live count.
struct SortScratch {
  int* off;
  int* sums;
  int* live;
};

// ranked: the counters and ranks are already there (grpic_push_deposit_ranked)
template <class T>
grpic_status sort_impl(grpic_ctx* c, const grpic_particles* src, const grpic_particles* dst, const SortScratch& w,
                       bool ranked, hipStream_t s) {
  const Grid& g = c->g;
  const int64_t nkeys = (int64_t)g.n_r * g.n_th + 1;
  const int nb = (int)((nkeys + kScanBlock - 1) / kScanBlock);
  const ParticleArraysT<T> a = arrays<T>(src), b = arrays<T>(dst);
  if (!ranked) {
    const dim3 grank((unsigned)((src->n + kRankBlock - 1) / kRankBlock));
    hipLaunchKernelGGL(sort_rank_kernel<T>, grank, dim3(kB), 0, s, g, a, w.off);
    LAUNCH_CHECK("sort_rank");
  }
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(nb), dim3(256), 0, s, w.off, nkeys, w.sums);
  LAUNCH_CHECK("scan_blocks");
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, s, w.sums, nb);
  LAUNCH_CHECK("scan_sums");
  hipLaunchKernelGGL(scan_add_kernel, dim3(blocks(nkeys)), dim3(kB), 0, s, w.off, nkeys, w.sums);
  LAUNCH_CHECK("scan_add");
  hipLaunchKernelGGL(copy_int_kernel, dim3(1), dim3(1), 0, s, w.off + (nkeys - 1), w.live);
  LAUNCH_CHECK("copy_int");
  hipLaunchKernelGGL(sort_scatter_kernel<T>, dim3(blocks(src->n)), dim3(kB), 0, s, g, a, b, (const int*)w.off);
  LAUNCH_CHECK("sort_scatter");
  hipLaunchKernelGGL(sort_clear_tail_kernel, dim3(1024), dim3(kB), 0, s, b.tag, dst->n, (const int*)w.live);
  LAUNCH_CHECK("sort_clear_tail");
  return GRPIC_OK;
}

grpic_status sort_check(grpic_ctx* c, const grpic_particles* src, const grpic_particles* dst) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_particles(src)) || (st = check_particles(dst))) return st;
  if (src->n != dst->n) return fail(GRPIC_EINVAL, "source has %lld slots, destination %lld",
                                    (long long)src->n, (long long)dst->n);
  if (src->n > 0x7FFFFFFFll) return fail(GRPIC_EINVAL, "more than 2^31 - 1 slots");
  if (src->n > 0 && (src->tag == dst->tag || src->u1 == dst->u1))
    return fail(GRPIC_EINVAL, "source and destination must not alias");
  return GRPIC_OK;
}

// Argument checks and the launch sequence of a sort into the given scratch
// (counters cleared by a fill kernel first, unless `ranked`: then the
// scratch holds the counters of grpic_push_deposit_ranked).
grpic_status sort_run(grpic_ctx* c, const grpic_particles* src, const grpic_particles* dst, const SortScratch& w,
                      hipStream_t s, bool ranked = false) {
  grpic_status st;
  if ((st = sort_check(c, src, dst))) return st;
  const Grid& g = c->g;
  const int64_t nkeys = (int64_t)g.n_r * g.n_th + 1;
  if (!ranked) {
    hipLaunchKernelGGL(fill_int_kernel, dim3(blocks(nkeys)), dim3(kB), 0, s, nkeys, w.off, 0);
    LAUNCH_CHECK("fill_int");
  }
  if (src->n > 0) {
    if ((st = c->f32 ? sort_impl<float>(c, src, dst, w, ranked, s) : sort_impl<double>(c, src, dst, w, ranked, s)))
      return st;
  } else {
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, s, (int64_t)1, w.live, 0);
    LAUNCH_CHECK("fill_int");
  }
  return GRPIC_OK;
}

// This device's address of `scratch`, looked up once per device (with that
// device current) and kept for the process.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int* g_scratch_ptr[kMaxDevices] = {};

grpic_status static_scratch_of(int device, int** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return fail(GRPIC_EINVAL, "device %d out of range", device);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(GRPIC_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<int*>(p);
  }
  *out = g_scratch_ptr[device];
  return GRPIC_OK;
}

template <class T, bool kQ>
grpic_status field_advance_impl(grpic_ctx* c, const grpic_fields* F, int32_t stage, hipStream_t s) {
  grpic_status st;
  const Grid& g = c->g;
  const dim3 gaux = grid2(g.n_r + 2, g.n_th + 1);   // i in [-1, n_r], j in [0, n_th]
  const dim3 gupd = grid2(g.n_r + 1, g.n_th + 1);   // i in [0, n_r],  j in [0, n_th]
  const dim3 gpl2 = grid2(g.n_r + 2 * g.ng, g.n_th + 2 * g.ng);  // whole plane
  if (stage == GRPIC_FIELDS_PRE_PUSH) {
    // B0 <- (B0 + B)/2, D0 <- (D0 + D)/2; E from (B, D0); B0 += Faraday(E)
    hipLaunchKernelGGL(average_kernel<T>, dim3(blocks(g.plane)), dim3(kB), 0, s, g.plane, tri<T>(F->B0),
                       ctri<T>(F->B), tri<T>(F->D0), ctri<T>(F->D));
    LAUNCH_CHECK("average");
    hipLaunchKernelGGL((aux_kernel<T, true, false, kQ>), gaux, kBlock2, 0, s, g, c->tab, ctri<T>(F->B),
                       ctri<T>(F->D0), tri<T>(F->E), none<T>());
    LAUNCH_CHECK("aux_e");
    hipLaunchKernelGGL((faraday_kernel<T, false, kQ>), gupd, kBlock2, 0, s, g, c->tab, tri<T>(F->B0), none<T>(),
                       ctri<T>(F->E), none<T>());
    LAUNCH_CHECK("faraday");
    return field_bc<T>(c, tri<T>(F->B0), none<T>(), ctri<T>(F->Binit), true, s);
  }
  // current filter (n_f passes) on the freshly deposited J^{n+1/2}, T as the
  // second plane set
  TriT<T> Jf;  // the filtered current: J itself, or the scratch set T
  if ((st = filter_passes<T>(c, tri<T>(F->J), tri<T>(F->T), 3, kStagD2, int3{1, -1, -1}, s, &Jf))) return st;
  const TriT<T> Jclear = Jf.p[0] == (T*)F->J[0] ? none<T>() : tri<T>(F->J);
  // E, H from (B0, D); B0 <- B and B += Faraday(E)
  hipLaunchKernelGGL((aux_kernel<T, true, true, kQ>), gaux, kBlock2, 0, s, g, c->tab, ctri<T>(F->B0),
                     ctri<T>(F->D), tri<T>(F->E), tri<T>(F->H));
  LAUNCH_CHECK("aux_eh");
  hipLaunchKernelGGL((faraday_kernel<T, true, kQ>), gpl2, kBlock2, 0, s, g, c->tab, tri<T>(F->B), comp<T>(c, F->Bc),
                     ctri<T>(F->E), tri<T>(F->B0));
  LAUNCH_CHECK("faraday");
  if ((st = field_bc<T>(c, tri<T>(F->B), comp<T>(c, F->Bc), ctri<T>(F->Binit), true, s))) return st;
  // D0 += Ampere(H, (J0 + J)/2)
  hipLaunchKernelGGL((ampere_kernel<T, false, kQ>), gupd, kBlock2, 0, s, g, c->tab, tri<T>(F->D0), none<T>(),
                     ctri<T>(F->H), tri<T>(F->J0), Jf, 0.5, 0.5, c->polar_k, none<T>(), none<T>());
  LAUNCH_CHECK("ampere");
  if ((st = field_bc<T>(c, tri<T>(F->D0), none<T>(), ctri<T>(F->Dinit), false, s))) return st;
  // H from (B, D0); D0 <- D, D += Ampere(H, J), J0 <- J, J <- 0
  hipLaunchKernelGGL((aux_kernel<T, false, true, kQ>), gaux, kBlock2, 0, s, g, c->tab, ctri<T>(F->B),
                     ctri<T>(F->D0), none<T>(), tri<T>(F->H));
  LAUNCH_CHECK("aux_h");
  hipLaunchKernelGGL((ampere_kernel<T, true, kQ>), gpl2, kBlock2, 0, s, g, c->tab, tri<T>(F->D), comp<T>(c, F->Dc),
                     ctri<T>(F->H), Jf, tri<T>(F->J0), 1.0, 0.0, c->polar_k, tri<T>(F->D0), Jclear);
  LAUNCH_CHECK("ampere");
  return field_bc<T>(c, tri<T>(F->D), comp<T>(c, F->Dc), ctri<T>(F->Dinit), false, s);
}

template <class T>
grpic_status inject_impl(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P, const InjectArgs& a,
                         hipStream_t s) {
  const Grid& g = c->g;
  const int64_t ncell = (int64_t)g.n_r * g.n_th, nkeys = ncell + 1;
  const int nb = (int)((nkeys + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(fill_kernel<double>, dim3(blocks(ncell)), dim3(kB), 0, s, ncell, c->inj_w, 0.0);
  LAUNCH_CHECK("fill");
  if (P->n > 0) {
    hipLaunchKernelGGL(inject_weights_kernel<T>, dim3(blocks(P->n)), dim3(kB), 0, s, g, arrays<T>(P), c->inj_w);
    LAUNCH_CHECK("inject_weights");
  }
  hipLaunchKernelGGL(inject_cells_kernel<T>, dim3(blocks(nkeys)), dim3(kB), 0, s, g, c->tab, (const T*)F->B[0],
                     (const T*)F->B[1], (const T*)F->B[2], (const double*)c->inj_w, a, c->sort_off);
  LAUNCH_CHECK("inject_cells");
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(nb), dim3(256), 0, s, c->sort_off, nkeys, c->sort_sums);
  LAUNCH_CHECK("scan_blocks");
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, s, c->sort_sums, nb);
  LAUNCH_CHECK("scan_sums");
  hipLaunchKernelGGL(scan_add_kernel, dim3(blocks(nkeys)), dim3(kB), 0, s, c->sort_off, nkeys, c->sort_sums);
  LAUNCH_CHECK("scan_add");
  hipLaunchKernelGGL(inject_pairs_kernel<T>, dim3(blocks(ncell)), dim3(kB), 0, s, g, arrays<T>(P),
                     (const int*)c->sort_off, a);
  LAUNCH_CHECK("inject_pairs");
  return GRPIC_OK;
}

template <class T>
grpic_status diagnostics_impl(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P, double B0,
                              void* E_out, void* L_out, void* gauss_res, hipStream_t s) {
  const Grid& g = c->g;
  if (P->n > 0) {
    const dim3 gd(std::min(blocks(P->n), (unsigned)kDiagMaxBlocks)), bd(kDiagBlock);
    switch (g.ser) {
      case 2: hipLaunchKernelGGL((diag_particles_kernel<T, 2>), gd, bd, 0, s, g, c->tab, arrays<T>(P), B0, (T*)E_out, (T*)L_out, c->acc); break;
      case 1: hipLaunchKernelGGL((diag_particles_kernel<T, 1>), gd, bd, 0, s, g, c->tab, arrays<T>(P), B0, (T*)E_out, (T*)L_out, c->acc); break;
      default: hipLaunchKernelGGL((diag_particles_kernel<T, 0>), gd, bd, 0, s, g, c->tab, arrays<T>(P), B0, (T*)E_out, (T*)L_out, c->acc); break;
    }
    LAUNCH_CHECK("diag_particles");
  }
  // Gauss residual: charge into T[0], filtered like the currents (T[1] scratch)
  T* Q = (T*)F->T[0];
  T* tmp = (T*)F->T[1];
  hipLaunchKernelGGL(fill_kernel<T>, dim3(blocks(g.plane)), dim3(kB), 0, s, g.plane, Q, 0.0);
  LAUNCH_CHECK("fill");
  if (P->n > 0) {
    hipLaunchKernelGGL(charge_kernel<T>, dim3(blocks(P->n)), dim3(kB), 0, s, g, arrays<T>(P), Q);
    LAUNCH_CHECK("charge");
  }
  {
    grpic_status st;
    TriT<T> A{{Q, nullptr, nullptr}}, B{{tmp, nullptr, nullptr}}, out;
    if ((st = filter_passes<T>(c, A, B, 1, int3{0, 0, 0}, int3{1, 1, 1}, s, &out))) return st;
    Q = out.p[0];
  }
  if (gauss_res) {
    hipLaunchKernelGGL(fill_kernel<T>, dim3(blocks(g.plane)), dim3(kB), 0, s, g.plane, (T*)gauss_res, 0.0);
    LAUNCH_CHECK("fill");
  }
  const int i_hi = g.n_r - std::max(g.n_absorb, g.n_filter);
  const int ni = i_hi - (g.n_filter + 2), nj = g.n_th + 1;
  if (ni > 0) {
    if (g.r0 != 0.0 || g.h0 != 0.0)
      hipLaunchKernelGGL((gauss_kernel<T, true>), grid2(ni, nj), kBlock2, 0, s, g, c->tab, c->polar_k, i_hi,
                         (const T*)F->D[0], (const T*)F->D[1], (const T*)Q, (T*)gauss_res, c->acc);
    else
      hipLaunchKernelGGL((gauss_kernel<T, false>), grid2(ni, nj), kBlock2, 0, s, g, c->tab, c->polar_k, i_hi,
                         (const T*)F->D[0], (const T*)F->D[1], (const T*)Q, (T*)gauss_res, c->acc);
    LAUNCH_CHECK("gauss");
  }
  return GRPIC_OK;
}

}  // namespace

extern "C" {

const char* grpic_last_error(void) { return g_err.c_str(); }

// Calls that change a particle set end the validity of the ranks of
// grpic_push_deposit_ranked (the next grpic_sort_ranked then fails).
inline void drop_ranks(grpic_ctx* c) {
  if (c) c->ranked = false;
}

grpic_status grpic_create(const grpic_params* p, grpic_ctx** out) {
  if (!p || !out) return fail(GRPIC_EINVAL, "null argument");
  *out = nullptr;
  if (p->precision != GRPIC_FP64 && p->precision != GRPIC_FP32)
    return fail(GRPIC_EINVAL, "unknown precision %d", p->precision);
  if (p->n_r < 8 || p->n_th < 8) return fail(GRPIC_EINVAL, "grid %d x %d too small", p->n_r, p->n_th);
  if (p->n_ghost != 2) return fail(GRPIC_EINVAL, "n_ghost must be 2 (got %d)", p->n_ghost);
  if (p->n_iter < 1) return fail(GRPIC_EINVAL, "n_iter must be >= 1");
  if (p->n_filter < 0 || p->n_absorb < 0) return fail(GRPIC_EINVAL, "negative n_filter or n_absorb");
  if (p->n_filter + 2 >= p->n_r - p->n_absorb)
    return fail(GRPIC_EINVAL, "boundary layers overlap (n_filter %d, n_absorb %d, n_r %d)", p->n_filter,
                p->n_absorb, p->n_r);
  if (!(p->r_min > 0.0) || !(p->r_max > p->r_min)) return fail(GRPIC_EINVAL, "need 0 < r_min < r_max");
  if (!(p->r0 >= 0.0 && p->r0 < p->r_min)) return fail(GRPIC_EINVAL, "need 0 <= r0 < r_min");
  if (!(p->h0 > -0.5 && p->h0 < 1.0)) return fail(GRPIC_EINVAL, "need -1/2 < h0 < 1");
  if (!((p->M > 0.0 && std::fabs(p->a) < p->M) || (p->M == 0.0 && p->a == 0.0)))
    return fail(GRPIC_EINVAL, "need |a| < M (or M = a = 0)");
  if (!(p->small_angle > 0.0 && p->small_angle < 0.1)) return fail(GRPIC_EINVAL, "small_angle out of range");
  if (p->reserved != 0) return fail(GRPIC_EINVAL, "reserved must be 0");
  if (!(p->iter_tol >= 0.0 && p->iter_tol < 1e-6)) return fail(GRPIC_EINVAL, "iter_tol must be in [0, 1e-6)");
  if ((int64_t)(p->n_r + 2 * p->n_ghost) * (p->n_th + 2 * p->n_ghost) > (int64_t)1 << 31)
    return fail(GRPIC_EINVAL, "grid too large");

  grpic_ctx* c = new grpic_ctx();
  c->prm = *p;
  c->f32 = p->precision == GRPIC_FP32;
  Grid& g = c->g;
  g.a = p->a;
  g.M = p->M;
  g.a2 = g.a * g.a;
  g.two_M = 2.0 * g.M;
  g.th_hi = kPi - p->small_angle;
  g.r0 = p->r0;
  g.h0 = p->h0;
  g.xi_min = std::log(p->r_min - p->r0);
  g.dxi = std::log((p->r_max - p->r0) / (p->r_min - p->r0)) / p->n_r;
  g.dth = kPi / p->n_th;
  g.inv_dth2 = 1.0 / (g.dth * g.dth);
  g.small_angle = p->small_angle;
  g.charge_scale = p->charge_scale;
  g.iter_tol = p->iter_tol;
  g.n_r = p->n_r;
  g.n_th = p->n_th;
  g.ng = p->n_ghost;
  g.ld = p->n_th + 2 * p->n_ghost;
  g.n_iter = p->n_iter;
  g.n_filter = p->n_filter;
  g.n_absorb = p->n_absorb;
  g.plane = (int64_t)(p->n_r + 2 * p->n_ghost) * g.ld;
  if (p->dt > 0.0) {
    g.dt = p->dt;
  } else {
    if (!(p->cfl > 0.0)) {
      delete c;
      return fail(GRPIC_EINVAL, "dt <= 0 needs cfl > 0");
    }
    // Courant rule over the cell centres (host evaluation)
    double vmax = 0.0;
    for (int i = 0; i < p->n_r; ++i)
      for (int j = 0; j < p->n_th; ++j) {
        const Coeffs m = coeffs_at(g, i + 0.5, j + 0.5);
        const double v1 = m.alpha * std::sqrt(m.hu11) + std::fabs(m.beta1);
        const double v2 = m.alpha * std::sqrt(m.hu22);
        vmax = std::fmax(vmax, std::sqrt(v1 * v1 + v2 * v2));
      }
    g.dt = p->cfl / vmax;
  }
  c->prm.dt = g.dt;
  {
    // the polar cap of the axis update ends at theta(x2 = 1/2)
    double thc, td, dtd;
    map_theta(g, 0.5, &thc, &td, &dtd);
    c->polar_k = 1.0 - std::cos(thc);
  }
  g.sin_lo = std::sin(p->small_angle);
  g.cos_lo = std::cos(p->small_angle);
  g.sin_hi = std::sin(kPi - p->small_angle);
  g.cos_hi = std::cos(kPi - p->small_angle);
  // the push evaluates exp and sincos of in-cell offsets (at most 1.5 cells)
  // by series that are exact to rounding for arguments up to 0.03 (short) or
  // 0.11 (long)
  // (the series are written for the logarithmic-r, uniform-theta grid; a
  // general quasi-spherical map takes the library functions)
  {
    const double off = 1.5 * std::fmax(g.dxi, g.dth);
    g.ser = (off <= 0.03 && 4.0 * g.dth <= 0.03) ? 2 : (off <= 0.11 ? 1 : 0);
    g.axis_band = 4.0 * g.dth;
    g.band_hi = kPi - g.axis_band;
    if (g.r0 != 0.0 || g.h0 != 0.0) g.ser = 0;
  }
  // single-precision push: cells whose inner edge lies below r = 3 M keep the
  // metric and its derivatives in FP64 (the horizon region, where lapse and
  // shift vary fastest)
  g.i_fp64 = 0;
  if (g.M > 0.0 && 3.0 * g.M > g.r0) {
    const double x = std::ceil((std::log(3.0 * g.M - g.r0) - g.xi_min) / g.dxi);
    g.i_fp64 = (int)std::fmin(std::fmax(x, 0.0), (double)p->n_r);
  }

  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) {
    grpic_status sst = static_scratch_of(c->device, &c->static_scratch);
    if (sst != GRPIC_OK) {
      delete c;
      return sst;
    }
  }
  const int nr = p->n_r + 2 * p->n_ghost, nt = p->n_th + 2 * p->n_ghost;
  // r, 1/(R deta); sin, cos, 1/sin, T = dtheta/dx2, deta/T (integer, half-integer)
  const size_t nt_all = 4 * (size_t)nr + 10 * (size_t)nt;
  const size_t nf_all = (size_t)nr + 2 * (size_t)nt;  // float r - r0, sin, cos at integer nodes
  const size_t bytes = nt_all * sizeof(double) + nf_all * sizeof(float);
  if (e == hipSuccess) e = hipMalloc(&c->tables, bytes);
  if (e != hipSuccess) {
    delete c;
    return fail(GRPIC_ENOMEM, "table allocation: %s", hipGetErrorString(e));
  }
  e = hipMalloc(&c->acc, sizeof(DiagAcc));
  if (e != hipSuccess) {
    (void)hipFree(c->tables);
    delete c;
    return fail(GRPIC_ENOMEM, "accumulator allocation: %s", hipGetErrorString(e));
  }
  {
    const int64_t nkeys = (int64_t)p->n_r * p->n_th + 1;
    const int64_t nb = (nkeys + kScanBlock - 1) / kScanBlock;
    e = hipMalloc(&c->sort_off, (nkeys + nb + 1) * sizeof(int));
    if (e != hipSuccess) {
      (void)hipFree(c->tables);
      (void)hipFree(c->acc);
      delete c;
      return fail(GRPIC_ENOMEM, "sort scratch allocation: %s", hipGetErrorString(e));
    }
    c->sort_sums = c->sort_off + nkeys;
    c->sort_live = c->sort_sums + nb;
  }
  double* h = new double[(bytes + sizeof(double) - 1) / sizeof(double)];
  // layout: r[2], ird[2] (nr each); s[2], c[2], is[2], td[2], eta_t[2] (nt each)
  double* tr[2] = {h, h + nr};
  double* tird[2] = {h + 2 * nr, h + 3 * nr};
  double* ts[2] = {h + 4 * nr, h + 4 * nr + nt};
  double* tc[2] = {ts[1] + nt, ts[1] + 2 * nt};
  double* tis[2] = {tc[1] + nt, tc[1] + 2 * nt};
  double* ttd[2] = {tis[1] + nt, tis[1] + 2 * nt};
  double* tet[2] = {ttd[1] + nt, ttd[1] + 2 * nt};
  for (int o = 0; o < 2; ++o) {
    for (int i = 0; i < nr; ++i) {
      double rd;
      map_r(g, (double)(i - g.ng) + 0.5 * o, &tr[o][i], &rd);
      tird[o][i] = 1.0 / (rd * g.dth);
    }
    for (int j = 0; j < nt; ++j) {
      double th, dtd;
      map_theta(g, (double)(j - g.ng) + 0.5 * o, &th, &ttd[o][j], &dtd);
      ts[o][j] = std::sin(th);
      tc[o][j] = std::cos(th);
      const bool axis = o == 0 && (j == g.ng || j == g.ng + p->n_th);
      tis[o][j] = axis ? 0.0 : 1.0 / ts[o][j];  // no inverse on the axis
      tet[o][j] = g.dth / ttd[o][j];
    }
  }
  float* hf = reinterpret_cast<float*>(h + nt_all);
  for (int i = 0; i < nr; ++i) hf[i] = (float)(tr[0][i] - g.r0);
  for (int j = 0; j < nt; ++j) {
    hf[nr + j] = (float)ts[0][j];
    hf[nr + nt + j] = (float)tc[0][j];
  }
  for (int o = 0; o < 2; ++o) {
    c->tab.r[o] = c->tables + (tr[o] - h);
    c->tab.ird[o] = c->tables + (tird[o] - h);
    c->tab.s[o] = c->tables + (ts[o] - h);
    c->tab.c[o] = c->tables + (tc[o] - h);
    c->tab.is[o] = c->tables + (tis[o] - h);
    c->tab.td[o] = c->tables + (ttd[o] - h);
    c->tab.eta_t[o] = c->tables + (tet[o] - h);
  }
  e = hipMemcpy(c->tables, h, bytes, hipMemcpyHostToDevice);
  delete[] h;
  if (e != hipSuccess) {
    (void)hipFree(c->tables);
    (void)hipFree(c->acc);
    (void)hipFree(c->sort_off);
    delete c;
    return fail(GRPIC_EHIP, "table upload: %s", hipGetErrorString(e));
  }
  const float* tf = reinterpret_cast<const float*>(c->tables + nt_all);
  c->tab.rf = tf;
  c->tab.sf = tf + nr;
  c->tab.cf = tf + nr + nt;
  *out = c;
  return GRPIC_OK;
}

grpic_status grpic_destroy(grpic_ctx* c) {
  if (!c) return GRPIC_OK;
  (void)hipFree(c->tables);
  (void)hipFree(c->acc);
  (void)hipFree(c->sort_off);
  if (c->inj_w) (void)hipFree(c->inj_w);
  if (c->rank_off) (void)hipFree(c->rank_off);
  delete c;
  return GRPIC_OK;
}

grpic_status grpic_get_params(const grpic_ctx* c, grpic_params* out) {
  if (!c || !out) return fail(GRPIC_EINVAL, "null argument");
  *out = c->prm;
  return GRPIC_OK;
}

grpic_status grpic_particles_init(grpic_ctx* c, const grpic_particles* P, int64_t n_pairs,
                                  int32_t ppc, double T, int64_t n_geo, uint64_t seed, void* stream) {
  drop_ranks(c);
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_particles(P))) return st;
  const Grid& g = c->g;
  if (ppc < 0 || (ppc % 2) != 0) return fail(GRPIC_EINVAL, "ppc must be even and >= 0 (got %d)", ppc);
  if (ppc > 0) n_pairs = (int64_t)g.n_r * g.n_th * (ppc / 2);
  if (n_pairs < 0 || n_geo < 0) return fail(GRPIC_EINVAL, "negative counts");
  if (!(T > 0.0)) return fail(GRPIC_EINVAL, "temperature must be > 0");
  if (2 * n_pairs + n_geo != P->n)
    return fail(GRPIC_ECAPACITY, "particle set has %lld slots, request needs %lld", (long long)P->n,
                (long long)(2 * n_pairs + n_geo));
  if (2 * n_pairs + n_geo > 0xFFFFFFFFll) return fail(GRPIC_EINVAL, "more than 2^32 particles");
  if (n_geo > 0 && !(6.0 > c->prm.r_min && 15.0 < c->prm.r_max && g.M > 0.0))
    return fail(GRPIC_EINVAL, "test geodesics need r in [6, 15] inside the grid and M > 0");
  return c->f32 ? particles_init_impl<float>(c, P, n_pairs, ppc, T, n_geo, seed, S(stream))
                : particles_init_impl<double>(c, P, n_pairs, ppc, T, n_geo, seed, S(stream));
}

grpic_status grpic_fields_init_monopole(grpic_ctx* c, const grpic_fields* F, double B0, void* stream) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F))) return st;
  return c->f32 ? monopole_impl<float>(c, F, B0, S(stream)) : monopole_impl<double>(c, F, B0, S(stream));
}

grpic_status grpic_fields_init_wald(grpic_ctx* c, const grpic_fields* F, double B0, void* stream) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F))) return st;
  return c->f32 ? wald_impl<float>(c, F, B0, S(stream)) : wald_impl<double>(c, F, B0, S(stream));
}

grpic_status grpic_push(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P, void* stream) {
  drop_ranks(c);
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F)) || (st = check_particles(P))) return st;
  if (P->n == 0) return GRPIC_OK;
  return push_impl(c, F, P, S(stream));
}

grpic_status grpic_deposit(grpic_ctx* c, const grpic_particles* P, const grpic_fields* F, void* stream) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F)) || (st = check_particles(P))) return st;
  if (P->n == 0) return GRPIC_OK;
  return c->f32 ? deposit_impl<float>(c, P, F, S(stream)) : deposit_impl<double>(c, P, F, S(stream));
}

grpic_status grpic_push_deposit(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P,
                                void* stream) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F)) || (st = check_particles(P))) return st;
  c->ranked = false;
  if (P->n == 0) return GRPIC_OK;
  return push_deposit_impl(c, F, P, nullptr, S(stream));
}

grpic_status grpic_push_deposit_ranked(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P,
                                       void* stream) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F)) || (st = check_particles(P))) return st;
  if (P->n > 0x7FFFFFFFll) return fail(GRPIC_EINVAL, "more than 2^31 - 1 slots");
  c->ranked = false;
  const int64_t nkeys = (int64_t)c->g.n_r * c->g.n_th + 1;
  const int64_t nb = (nkeys + kScanBlock - 1) / kScanBlock;
  if (!c->rank_off) {
    const hipError_t e = hipMalloc(&c->rank_off, (nkeys + nb + 1) * sizeof(int));
    if (e != hipSuccess) {
      c->rank_off = nullptr;
      return fail(GRPIC_ENOMEM, "rank scratch allocation: %s", hipGetErrorString(e));
    }
  }
  hipStream_t s = S(stream);
  hipLaunchKernelGGL(fill_int_kernel, dim3(blocks(nkeys)), dim3(kB), 0, s, nkeys, c->rank_off, 0);
  LAUNCH_CHECK("fill_int");
  if (P->n > 0 && (st = push_deposit_impl(c, F, P, c->rank_off, s))) return st;
  c->ranked = true;
  c->ranked_i1p = P->i1p;
  c->ranked_n = P->n;
  return GRPIC_OK;
}

grpic_status grpic_push_adjoint(grpic_ctx* c, const grpic_fields* F, double B0, const grpic_particles* P,
                                const double* gbar_in, double* gbar_out, double* gbar_B0, void* stream) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F)) || (st = check_particles(P))) return st;
  if (c->f32) return fail(GRPIC_ESTATE, "the adjoint needs a GRPIC_FP64 context");
  if (!(B0 != 0.0 && std::isfinite(B0))) return fail(GRPIC_EINVAL, "B0 must be finite and non-zero");
  if (P->n == 0) return GRPIC_OK;
  if (!gbar_in || !gbar_out || !gbar_B0) return fail(GRPIC_EINVAL, "null adjoint array");
  GatherPlanesT<double> gp;
  for (int k = 0; k < 3; ++k) {
    gp.D[k] = (const double*)F->D[k];
    gp.B[k] = (const double*)F->B0[k];
  }
  hipLaunchKernelGGL(push_adjoint_kernel, dim3((unsigned)((P->n + 63) / 64)), dim3(64), 0, S(stream), c->g, gp,
                     1.0 / B0, arrays<double>(P), gbar_in, gbar_out, gbar_B0);
  LAUNCH_CHECK("push_adjoint");
  return GRPIC_OK;
}

grpic_status grpic_sort(grpic_ctx* c, const grpic_particles* src, const grpic_particles* dst,
                        int64_t* n_live, void* stream) {
  drop_ranks(c);
  grpic_status st;
  hipStream_t s = S(stream);
  if (!c) return fail(GRPIC_EINVAL, "null context");
  if ((st = sort_run(c, src, dst, SortScratch{c->sort_off, c->sort_sums, c->sort_live}, s))) return st;
  if (n_live) {
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, c->sort_live, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_live = h;
  }
  return GRPIC_OK;
}

grpic_status grpic_sort_ranked(grpic_ctx* c, const grpic_particles* src, const grpic_particles* dst,
                               int64_t* n_live, void* stream) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_particles(src))) return st;
  if (!c->rank_off || !c->ranked || c->ranked_i1p != src->i1p || c->ranked_n != src->n)
    return fail(GRPIC_ESTATE, "no grpic_push_deposit_ranked of this particle set since its last change");
  const int64_t nkeys = (int64_t)c->g.n_r * c->g.n_th + 1;
  const int64_t nb = (nkeys + kScanBlock - 1) / kScanBlock;
  hipStream_t s = S(stream);
  const SortScratch w{c->rank_off, c->rank_off + nkeys, c->rank_off + nkeys + nb};
  if ((st = sort_run(c, src, dst, w, s, true))) return st;
  c->ranked = false;
  if (n_live) {
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, w.live, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_live = h;
  }
  return GRPIC_OK;
}

grpic_status grpic_sort_noalloc(grpic_ctx* c, const grpic_particles* src, const grpic_particles* dst,
                                int32_t* n_live_device, void* stream) {
  drop_ranks(c);
  grpic_status st;
  if (!c) return fail(GRPIC_EINVAL, "null context");
  const int64_t ncell = (int64_t)c->g.n_r * c->g.n_th;
  if (ncell > kStaticSortCells)
    return fail(GRPIC_EINVAL, "grid of %lld cells exceeds the static sort scratch (%lld cells)", (long long)ncell,
                (long long)kStaticSortCells);
  int* base = c->static_scratch;
  const int64_t nkeys = ncell + 1;
  const int64_t nb = (nkeys + kScanBlock - 1) / kScanBlock;
  hipStream_t s = S(stream);
  if ((st = sort_run(c, src, dst, SortScratch{base, base + nkeys, base + nkeys + nb}, s))) return st;
  if (n_live_device) {
    hipLaunchKernelGGL(copy_int_kernel, dim3(1), dim3(1), 0, s, (const int*)(base + nkeys + nb), n_live_device);
    LAUNCH_CHECK("copy_int");
  }
  return GRPIC_OK;
}

grpic_status grpic_inject_pairs(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P,
                                const grpic_inject_params* ip, int64_t first_free, int64_t* n_injected,
                                void* stream) {
  drop_ranks(c);
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F)) || (st = check_particles(P))) return st;
  if (!ip) return fail(GRPIC_EINVAL, "null injection parameters");
  if (!(ip->sigma_th > 0.0 && std::isfinite(ip->sigma_th))) return fail(GRPIC_EINVAL, "sigma_th must be > 0");
  if (!(ip->temperature > 0.0 && std::isfinite(ip->temperature)))
    return fail(GRPIC_EINVAL, "temperature must be > 0");
  if (!std::isfinite(ip->weight)) return fail(GRPIC_EINVAL, "weight must be finite");
  if (ip->n_pairs < 0) return fail(GRPIC_EINVAL, "n_pairs must be >= 0");
  if (ip->reserved != 0) return fail(GRPIC_EINVAL, "reserved must be 0");
  if (ip->call == 0xFFFFFFFFu) return fail(GRPIC_EINVAL, "call must be below 2^32 - 1");
  if (first_free < 0 || first_free > P->n) return fail(GRPIC_EINVAL, "first_free %lld outside [0, %lld]",
                                                      (long long)first_free, (long long)P->n);
  const Grid& g = c->g;
  const int64_t ncell = (int64_t)g.n_r * g.n_th;
  if ((int64_t)ip->n_pairs * ncell > INT_MAX) return fail(GRPIC_EINVAL, "n_pairs times the cells exceeds 2^31 - 1");
  if (P->n > 0xFFFFFFFFll) return fail(GRPIC_EINVAL, "more than 2^32 slots");
  if (!c->inj_w) {
    hipError_t e = hipMalloc(&c->inj_w, (size_t)ncell * sizeof(double));
    if (e != hipSuccess) {
      c->inj_w = nullptr;
      return fail(GRPIC_ENOMEM, "injection scratch allocation: %s", hipGetErrorString(e));
    }
  }
  InjectArgs a;
  a.sigma_th = ip->sigma_th;
  a.temp = ip->temperature;
  a.weight = ip->weight;
  a.n_pairs = ip->n_pairs;
  a.i_lo = std::max(ip->i_lo, 0);
  a.i_hi = std::min(ip->i_hi, g.n_r);
  a.seed = ip->seed;
  a.sub = ip->call + 1u;
  a.first_free = first_free;
  hipStream_t s = S(stream);
  if ((st = c->f32 ? inject_impl<float>(c, F, P, a, s) : inject_impl<double>(c, F, P, a, s))) return st;
  if (n_injected) {
    int total = 0;
    HIP_TRY(hipMemcpyAsync(&total, c->sort_off + ncell, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_injected = std::min<int64_t>(total, (P->n - first_free) / 2);
  }
  return GRPIC_OK;
}

grpic_status grpic_field_advance(grpic_ctx* c, const grpic_fields* F, int32_t stage, void* stream) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F))) return st;
  if (stage != GRPIC_FIELDS_PRE_PUSH && stage != GRPIC_FIELDS_POST_DEPOSIT)
    return fail(GRPIC_EINVAL, "unknown field stage %d", stage);
  const bool q = c->g.r0 != 0.0 || c->g.h0 != 0.0;
  if (c->f32)
    return q ? field_advance_impl<float, true>(c, F, stage, S(stream))
             : field_advance_impl<float, false>(c, F, stage, S(stream));
  return q ? field_advance_impl<double, true>(c, F, stage, S(stream))
           : field_advance_impl<double, false>(c, F, stage, S(stream));
}

grpic_status grpic_diagnostics(grpic_ctx* c, const grpic_fields* F, const grpic_particles* P, double B0,
                               grpic_diag* out, void* E_out, void* L_out, void* gauss_res, void* stream) {
  grpic_status st;
  if ((st = check_ctx(c)) || (st = check_fields(c, F)) || (st = check_particles(P))) return st;
  if (!out) return fail(GRPIC_EINVAL, "null output");
  hipStream_t s = S(stream);
  HIP_TRY(hipMemsetAsync(c->acc, 0, sizeof(DiagAcc), s));
  if ((st = c->f32 ? diagnostics_impl<float>(c, F, P, B0, E_out, L_out, gauss_res, s)
                   : diagnostics_impl<double>(c, F, P, B0, E_out, L_out, gauss_res, s)))
    return st;
  DiagAcc h;
  HIP_TRY(hipMemcpyAsync(&h, c->acc, sizeof(DiagAcc), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < 4; ++k) {
    out->n_alive[k] = (int64_t)h.counts[k];
    out->sum_E[k] = h.sums[k];
    out->sum_L[k] = h.sums[4 + k];
  }
  out->n_leaving = (int64_t)h.counts[4];
  out->n_empty = (int64_t)h.counts[5];
  out->n_nonfinite = (int64_t)h.counts[6];
  double gm, gs;
  std::memcpy(&gm, &h.gmax_bits, sizeof gm);
  std::memcpy(&gs, &h.gscale_bits, sizeof gs);
  out->gauss_max = gm;
  out->gauss_scale = gs;
  return GRPIC_OK;
}

}  // extern "C"
