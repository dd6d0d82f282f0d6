/*
 * grpic.h -- C ABI of libgrpic.so, the MI355X (gfx950) implementation of the
 * data-parallel hot path of a general-relativistic particle-in-cell step
 * (Galishnikova, Hakobyan, Philippov, Crinquand, "Entity II: General
 * Relativistic Module").
 *
 * Problem (Sec. 3): particles and fields on an axisymmetric (r, theta) grid,
 * uniform in the code coordinates of the quasi-spherical Kerr-Schild map of
 * App. A, x1 = ln((r - r0) / (r_min - r0)) / dxi and x2 = eta / deta with
 * theta(eta) of concentration h0 (r0 = h0 = 0: logarithmic r, uniform theta),
 * in the 3+1 split of the Kerr metric of mass M and spin a (Sec. 2.1, App. A).
 *
 * Conventions shared by every call
 *  - Every pointer inside grpic_fields / grpic_particles is a device pointer,
 *    owned by the caller (the library never allocates or frees caller memory).
 *    The library owns only what grpic_create allocates (per-context tables and
 *    scratch), released by grpic_destroy.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work on
 *    it and return without waiting, except where stated.
 *  - Return value: GRPIC_OK (0) or a negative grpic_status.  Argument errors
 *    are detected on the host before anything is enqueued; a failed kernel
 *    launch returns GRPIC_EHIP.  grpic_last_error() gives a message for the
 *    last failure on the calling thread.  No call throws.
 *  - Real-valued arrays are double when the context precision is GRPIC_FP64
 *    and float when it is GRPIC_FP32 (the precision form: int32 cell index plus
 *    single-precision offset, momenta, fields and currents).
 *
 * Field storage (Sec. 3.3.1 Yee staggering, Sec. 3.4 time levels): every
 * component is one plane of (n_r + 2 n_ghost) x (n_th + 2 n_ghost) reals,
 * element (i, j) at (i + n_ghost) * (n_th + 2 n_ghost) + (j + n_ghost); a
 * component staggered to i+1/2 or j+1/2 is stored at index i or j.
 * D^1 (i+1/2, j), D^2 (i, j+1/2), D^3 (i, j); B^1 (i, j+1/2), B^2 (i+1/2, j),
 * B^3 (i+1/2, j+1/2); E_i as D^i, H_i as B^i, J^i (conformal sqrt(h) J^i) as D^i.
 *
 * Particle storage (Sec. 3, code units): structure of arrays; position = cell
 * index (i1, i2) plus offset (dx1, dx2) in [0, 1); covariant code components
 * u_1 = u_r dr/dx1, u_2 = u_theta dth/dx2, u_3 = u_phi; previous position
 * (i1p, i2p, dx1p, dx2p): written by grpic_push for grpic_deposit (Sec. 3.2)
 * and read by grpic_diagnostics (time-centred E, L); grpic_push_deposit does
 * not write it (grpic_push_deposit_ranked writes the sort's ranks to i1p) and
 * grpic_sort does not carry it, so a step whose E, L are
 * wanted is taken with grpic_push and grpic_deposit (same particle state bit
 * for bit, same currents to rounding order).
 * tag: 0 = empty slot, 1 = positron (q/m = +1), 2 = electron (q/m = -1),
 * 3 = neutral test particle (q = 0); 7 = massless neutral particle (species 3
 * with bit 0x04: gamma = sqrt(h^ij u_i u_j) of Sec. 2.3, the EM stage
 * skipped; its momentum must be non-zero, else the update divides by zero and
 * the slot turns non-finite); bit 0x80 = left the domain this step
 * (deposited once more, emptied by the next push); tag 0x40 = dropped by a
 * bounds guard (a position outside the grid or a move of a cell or more,
 * which the deposit cannot represent), never used again and counted as
 * non-finite by grpic_diagnostics.
 */
#ifndef GRPIC_H
#define GRPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GRPIC_OK = 0,
  GRPIC_EINVAL = -1,    /* invalid argument (null pointer, size, layout) */
  GRPIC_EHIP = -2,      /* HIP runtime error (allocation, launch)        */
  GRPIC_ENOMEM = -3,    /* device allocation of context tables failed    */
  GRPIC_ESTATE = -4,    /* call not valid for this context               */
  GRPIC_ECAPACITY = -5  /* particle arrays too small for the request     */
} grpic_status;

typedef enum { GRPIC_FP64 = 0, GRPIC_FP32 = 1 } grpic_precision;

typedef enum {
  GRPIC_FIELDS_PRE_PUSH = 0,     /* Sec. 3.4 step 2: B^n for the push          */
  GRPIC_FIELDS_POST_DEPOSIT = 1  /* Sec. 3.4 steps 5-8: B^{n+1/2}, D^{n+1}     */
} grpic_field_stage;

/* Run parameters (code units, G = c = 1). */
typedef struct {
  double a;             /* black-hole spin, |a| < M                          */
  double M;             /* mass; M = 0 with a = 0 is flat space (App. A)     */
  double r_min, r_max;  /* radial extent; r_min inside the horizon           */
  double dt;            /* time step; <= 0: set from cfl by grpic_create     */
  double cfl;           /* Courant number used when dt <= 0                  */
  double small_angle;   /* theta clamp for metric evaluation (Sec. 3.3.2)   */
  double charge_scale;  /* deposited charge per unit particle weight          */
  double iter_tol;      /* 0: the implicit iterations run n_iter times (an
                           iterate that repeats exactly ends them early with
                           the same result); > 0: they also end once the FP64
                           change of an iterate is at most iter_tol times its
                           size (a convergence test; results then differ from
                           the fixed count by about iter_tol times the
                           contraction of the map)                          */
  int32_t n_r, n_th;    /* cells in r and theta, >= 8 each                   */
  int32_t n_ghost;      /* ghost cells per side; must be 2                   */
  int32_t n_iter;       /* implicit-midpoint iterations (Sec. 3.1), >= 1    */
  int32_t n_filter;     /* current filter passes n_f (Sec. 3.3.3)            */
  int32_t n_absorb;     /* outer absorbing-layer width in cells, >= 0        */
  int32_t precision;    /* grpic_precision                                   */
  int32_t reserved;     /* must be 0                                         */
  double r0;            /* quasi-spherical map (App. A): xi = log(r - r0) is
                           uniform in x1; 0 <= r0 < r_min                    */
  double h0;            /* equatorial concentration of the polar map
                           theta = eta + 2 h0 eta (pi - 2 eta)(pi - eta)/pi^2,
                           eta uniform in x2; -1/2 < h0 < 1.  r0 = h0 = 0 is
                           the logarithmic-r, uniform-theta grid, the only
                           one whose push takes in-cell series (others take
                           the library exp and sincos)                       */
} grpic_params;

/* Device pointers to the field planes (Sec. 3.4 storage):
 * D, B   = em   (D^n, B^{n-1/2});
 * D0, B0 = em0  (D^{n-1}, B^{n-3/2} at a step boundary; B0 holds B^n after
 *          the pre-push stage, which is what the push interpolates);
 * E, H   = aux; J = cur (J^{n+1/2}, accumulated by the deposit);
 * J0     = cur0 (J^{n-1/2}); Dinit, Binit = targets of the absorbing layer;
 * T      = scratch;
 * Dc, Bc = GRPIC_FP32 only (ignored, may be NULL, for GRPIC_FP64): low-order
 *          parts of D and B.  The time integration keeps D + Dc and B + Bc to
 *          about 48 bits and stores their rounding to float in D and B, which
 *          is what every other stage reads; grpic_fields_init_wald zeroes them.
 * The 33 (FP64) or 39 (FP32) planes may be separate allocations. */
typedef struct {
  void *D[3], *B[3], *D0[3], *B0[3], *E[3], *H[3], *J[3], *J0[3];
  void *Dinit[3], *Binit[3], *T[3];
  void *Dc[3], *Bc[3];
} grpic_fields;

typedef struct {
  int64_t n;            /* number of slots                                   */
  int32_t *i1, *i2;
  void *dx1, *dx2, *u1, *u2, *u3, *w, *phi;
  int32_t *i1p, *i2p;
  void *dx1p, *dx2p;
  uint8_t *tag;
} grpic_particles;

/* Summary filled by grpic_diagnostics. */
typedef struct {
  int64_t n_alive[4];   /* by species tag & 3 (index 0 unused; 3 counts the
                           massive and massless neutral slots together)      */
  int64_t n_leaving;    /* slots with the leaving bit                       */
  int64_t n_empty;      /* tag == 0                                          */
  int64_t n_nonfinite;  /* live slots with a non-finite offset or momentum   */
  double sum_E[4], sum_L[4];  /* sums of E and L by species (Sec. 2.3)      */
  double gauss_max;     /* max |div D - 4 pi rho| over the checked nodes     */
  double gauss_scale;   /* largest single term of that residual              */
} grpic_diag;

typedef struct grpic_ctx grpic_ctx;

/* Message for the last non-OK status on the calling thread. */
const char* grpic_last_error(void);

/* Creates a context for the current HIP device: validates *params, fixes dt
 * (Courant rule when params->dt <= 0: dt = cfl / max over cell centres of the
 * coordinate light speed sqrt((alpha sqrt(h^11) + |beta^1|)^2 + (alpha sqrt(h^22))^2)),
 * builds the 1-D coordinate tables on the device.  Synchronous. */
grpic_status grpic_create(const grpic_params* params, grpic_ctx** out);
grpic_status grpic_destroy(grpic_ctx* ctx);
/* Copies the parameters in use (dt filled in) to *out. */
grpic_status grpic_get_params(const grpic_ctx* ctx, grpic_params* out);

/* Particle loading (Sec. 4 problem setup; particles uniform in the code cell,
 * isotropic Maxwell-Juttner momenta at temperature T in the local tetrad
 * frame, u_i = e_i^hat u_hat, App. A tetrad).  Pairs k = 0 .. n_pairs-1 go to
 * slots 2k (e+) and 2k+1 (e-) at one position; with ppc > 0 (even) pair k sits
 * in cell k / (ppc/2) (cell = i1 * n_th + i2) and n_pairs = n_r n_th ppc / 2;
 * with ppc == 0 the cell is drawn uniformly.  Then n_geo neutral bound test
 * particles.  Random numbers: Philox4x32-10 keyed by seed.  P->n must equal
 * 2 n_pairs + n_geo (GRPIC_ECAPACITY otherwise). */
grpic_status grpic_particles_init(grpic_ctx* ctx, const grpic_particles* P, int64_t n_pairs,
                                  int32_t ppc, double T, int64_t n_geo, uint64_t seed,
                                  void* stream);

/* Wald vacuum field of amplitude B0 (Sec. 4.1.2, eq. Wald): B from the
 * discrete curl of A_mu (eq. EB-set), D from the analytic solution; fills D, B,
 * D0, B0, Dinit, Binit, zeroes E, H, J, J0, T (and Dc, Bc in GRPIC_FP32). */
grpic_status grpic_fields_init_wald(grpic_ctx* ctx, const grpic_fields* F, double B0,
                                    void* stream);

/* Monopole initial data of the BZ test (Sec. "BZ monopole", eq. for A_phi):
 * A_phi = -B0 cos(theta), so B^1 (B^r) is the discrete curl of A_3 (eq.
 * EB-set) and every other component, D included, is zero; fills D, B, D0, B0,
 * Dinit, Binit and zeroes the other planes, like grpic_fields_init_wald. */
grpic_status grpic_fields_init_monopole(grpic_ctx* ctx, const grpic_fields* F, double B0,
                                        void* stream);

/* Particle update of Sec. 3.1 (steps 1-11) for every slot: interpolate D (plane
 * D) and B (plane B0) to x^n, EM half push in the tetrad frame, implicit
 * geodesic momentum update, EM half push, implicit coordinate update, phi
 * update, axis reflection and removal at the radial boundaries (Sec. 3.3.3). */
grpic_status grpic_push(grpic_ctx* ctx, const grpic_fields* F, const grpic_particles* P,
                        void* stream);

/* Charge-conserving conformal current deposit (Sec. 3.2) from the previous to
 * the current positions, added into J (the caller zeroes J; the post-deposit
 * field stage does). */
grpic_status grpic_deposit(grpic_ctx* ctx, const grpic_particles* P, const grpic_fields* F,
                           void* stream);

/* grpic_push followed by grpic_deposit in one pass over the particles (same
 * arguments, same results up to rounding order): the deposit takes each move
 * from registers and J^3 from the push's own evaluation of the phi velocity
 * at the path midpoint (Sec. 3.1 step 10, Sec. 3.2); the previous-position
 * arrays are left as they were. */
grpic_status grpic_push_deposit(grpic_ctx* ctx, const grpic_fields* F, const grpic_particles* P,
                                void* stream);

/* grpic_push_deposit that also does the first pass of the cell sort (a
 * layout device, not part of the paper's method) on the state it leaves: per
 * block of the pass, the live slots are counted per cell, each live slot's
 * rank within its cell goes to P's i1p, and the cells' counts to scratch of
 * the context (n_r n_th + 1 counters, plus the scan's block sums, allocated
 * on the first call).  Complete the sort with grpic_sort_ranked on the same
 * particle set: the two give what grpic_push_deposit then grpic_sort give
 * (the particle state the same, the order within a cell unspecified).  At
 * most 2^31 - 1 slots (GRPIC_EINVAL).  P's previous-position arrays other
 * than i1p are left as they were.  Each block of the pass waits for its
 * cells' claims at its end: measured on MI355X, the double-precision pass at
 * 2048^2 with 90 particles per cell grows by a third of the separate rank
 * pass's time, while the single-precision pass at 4096^2 with 16 per cell
 * grows by more than that pass takes (grpic_sort is then the faster). */
grpic_status grpic_push_deposit_ranked(grpic_ctx* ctx, const grpic_fields* F, const grpic_particles* P,
                                       void* stream);

/* Adjoint of one grpic_push step in a frozen field (the differentiation form;
 * GRPIC_FP64 contexts only).  The particle state is s = (x1, x2, u1, u2, u3),
 * x = cell + offset; the field set F holds B0 times a fixed field F1 (planes D
 * and B0, as grpic_push reads them), B0 finite and non-zero.  For the step
 * s' = Phi(s, B0) of Sec. 3.1 steps 2-10 with the particle boundaries of
 * Sec. 3.3.3, starting from the state in P (as grpic_push would read it),
 * computes per particle
 *   gbar_out = (ds'/ds)^T gbar_in,   gbar_B0 += (ds'/dB0) . gbar_in.
 * The implicit momentum and coordinate stages are differentiated at their
 * fixed points (implicit-function theorem), so the forward pass must run its
 * iterations to convergence (n_iter large enough; they stop at an exact
 * repeat).  gbar_in, gbar_out: device arrays of 5 n doubles, rows x1, x2, u1,
 * u2, u3 (row c at offset c n); they may be the same array.  gbar_B0: n
 * doubles, accumulated.  Slots that the step does not move (empty, leaving,
 * dropped) pass gbar through unchanged.  P is not modified. */
grpic_status grpic_push_adjoint(grpic_ctx* ctx, const grpic_fields* F, double B0,
                                const grpic_particles* P, const double* gbar_in, double* gbar_out,
                                double* gbar_B0, void* stream);

/* Field stages of the PIC loop (Sec. 3.4): stage GRPIC_FIELDS_PRE_PUSH or
 * GRPIC_FIELDS_POST_DEPOSIT (grpic_field_stage). */
grpic_status grpic_field_advance(grpic_ctx* ctx, const grpic_fields* F, int32_t stage,
                                 void* stream);

/* Cell sort (a layout device, not part of the paper's method): writes the
 * live slots of src into dst ordered by cell c = i1 * n_th + i2; empty slots
 * and slots with the leaving bit (already deposited) are dropped, and dst's
 * slots after the live ones get tag 0 (their other arrays are left as they
 * were).  The order of particles within one cell is unspecified.  The
 * previous-position arrays of dst are left as they were, and src's i1p is
 * overwritten for the live slots (it holds each slot's rank within its cell
 * during the sort): call it after
 * the deposit that reads them, not between grpic_push and grpic_deposit.  src and dst must
 * have the same n and must not alias.  If n_live is non-null, waits for the
 * stream and stores the number of live slots (they occupy dst[0 .. n_live)).
 * Uses scratch owned by the context (n_r n_th + 1 counters). */
grpic_status grpic_sort(grpic_ctx* ctx, const grpic_particles* src, const grpic_particles* dst,
                        int64_t* n_live, void* stream);

/* The cell sort of src into dst (as grpic_sort: same arguments, results and
 * n_live) from the counts and ranks that the last grpic_push_deposit_ranked
 * of this context left for src; it skips the sort's own counting pass.
 * GRPIC_ESTATE if the last grpic_push_deposit_ranked of this context was not
 * on src (the same i1p array and n), or if a call that changes particles
 * (grpic_particles_init, grpic_push, grpic_push_deposit, grpic_sort,
 * grpic_sort_noalloc, grpic_inject_pairs, or an earlier grpic_sort_ranked)
 * came in between.  Changes to src made outside the library in between leave
 * the result unspecified; every write stays inside dst. */
grpic_status grpic_sort_ranked(grpic_ctx* ctx, const grpic_particles* src, const grpic_particles* dst,
                               int64_t* n_live, void* stream);

/* grpic_sort for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same sort, with the same kernels and results, whose scratch is a static
 * device array of the library instead of the context's (no hipMalloc, no
 * hipFree, no allocating library call).
 *  - Limit: grids of at most 2^24 cells (4096 x 4096); larger grids return
 *    GRPIC_EINVAL before anything is enqueued.  The array (2^24 + 16387 ints,
 *    64.1 MiB) is held on every GPU the library runs on until the process
 *    ends.
 *  - Every call on one GPU uses that GPU's one array: calls that overlap on
 *    one GPU (several streams, threads or contexts) race.  The counters are
 *    cleared by the call itself.
 *  - n_live_device: optional device int32; receives the number of live slots
 *    (enqueued, no wait), so the call never synchronises the stream.
 * Arguments and errors otherwise as grpic_sort. */
grpic_status grpic_sort_noalloc(grpic_ctx* ctx, const grpic_particles* src, const grpic_particles* dst,
                                int32_t* n_live_device, void* stream);

/* Parameters of grpic_inject_pairs. */
typedef struct {
  double sigma_th;      /* magnetisation threshold (the paper's runs: 1000 and
                           2000), > 0                                        */
  double temperature;   /* T of the injected pairs in units of m c^2 (the
                           paper's runs: 0.5), > 0                           */
  double weight;        /* weight of every injected particle                 */
  int32_t n_pairs;      /* pairs added per injecting cell per call, >= 0     */
  int32_t i_lo, i_hi;   /* radial cells i_lo <= i < i_hi may inject (clipped
                           to the grid)                                      */
  int32_t reserved;     /* must be 0                                         */
  uint64_t seed;        /* Philox4x32-10 key                                 */
  uint32_t call;        /* index of this injection call, < 2^32 - 1: counter
                           word 1 is call + 1 (0 is the initial loading's)   */
} grpic_inject_params;

/* Pair injection where the plasma is strongly magnetised (Sec. 4.4 and
 * Sec. 4.5: e+- pairs at temperature T are added wherever the magnetisation
 * sigma = B_i B^i / (4 pi n m) reaches a threshold).
 *  - sigma of cell (i, j) at its centre: B^1 and B^2 the means of the values
 *    on its two faces, B^3 its own value, all from plane B;
 *    B_i B^i = h_ij B^i B^j; n = charge_scale * (sum of the weights of the
 *    live, not leaving e+ and e- in the cell, any slot) / sqrt(h); m = 1.
 *    The cell injects when B_i B^i > 0 and B_i B^i >= 4 pi sigma_th n (FP64,
 *    also in the GRPIC_FP32 form), so a magnetised empty cell injects.
 *  - Every injecting cell, in the order c = i n_th + j, adds n_pairs pairs:
 *    pair k (counted over the call) fills slots first_free + 2k (e+, tag 1)
 *    and first_free + 2k + 1 (e-, tag 2) at one position (no net charge),
 *    offsets uniform in the cell, isotropic Maxwell-Juttner momenta at T in
 *    the local tetrad frame (as grpic_particles_init), the given weight,
 *    phi = 0, previous position = position.  Pairs that would not fit below
 *    P->n are not written (whole pairs only).  Random numbers: Philox4x32-10,
 *    key seed, counter (index, call + 1, stream, attempt).
 *  - The slots from first_free on must be empty (after grpic_sort they are
 *    from its n_live on); first_free in [0, P->n].
 *  - If n_injected is non-null, waits for the stream and stores the number of
 *    pairs written.
 *  - Uses the context's scratch: the cell sort's counters and one FP64 value
 *    per cell, allocated by the first call (GRPIC_ENOMEM if that fails).
 *    Calls on one context must not overlap on different streams. */
grpic_status grpic_inject_pairs(grpic_ctx* ctx, const grpic_fields* F, const grpic_particles* P,
                                const grpic_inject_params* params, int64_t first_free,
                                int64_t* n_injected, void* stream);

/* Diagnostics (Sec. 2.3 conserved E, L at the time-centred position, the
 * midpoint of the previous position recorded by the last grpic_push and the
 * current one; Gauss's law Sec. 3.2).  E_out, L_out: optional device arrays of P->n reals (NaN for
 * empty slots); gauss_res: optional device plane for the residual.  Waits for
 * the stream; fills *out. */
grpic_status grpic_diagnostics(grpic_ctx* ctx, const grpic_fields* F, const grpic_particles* P,
                               double B0, grpic_diag* out, void* E_out, void* L_out,
                               void* gauss_res, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GRPIC_H */
