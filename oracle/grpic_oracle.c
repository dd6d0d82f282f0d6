/*
 * grpic_oracle.c -- plain, slow FP64 CPU oracle of the GRPIC hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
 * leg of bench.py may load this library.  It shares no code, header, table or
 * constant generator with the HIP library; the two agree only on the plain
 * array layouts described below.
 *
 * What it computes (Galishnikova, Hakobyan, Philippov, Crinquand, "Entity II:
 * General Relativistic Module"):
 *   - the Kerr-Schild 3+1 metric in quasi-spherical code coordinates (App. A,
 *     "Quasi-spherical Kerr-Schild": xi = log(r - r0), theta(eta) with the
 *     equatorial concentration h0; r0 = h0 = 0 is log r, uniform theta) with
 *     the mass M as a parameter; M = 0, a = 0 is the flat "kerr_schild_0"
 *     metric (App. A, "Spherical Minkowski");
 *   - the orthonormal tetrad (App. A, matrix forms of e^i_hat and e_i^hat);
 *   - the particle update of Sec. 3.1 (steps 1-11): field interpolation,
 *     tetrad-frame Boris half pushes, implicit geodesic momentum iteration
 *     (eq. discretized-geodesic-u), implicit coordinate iteration
 *     (eq. discretized-geodesic-x), out-of-plane angle (eq. ...-x-phi),
 *     particle boundaries (Sec. 3.3.3);
 *   - the conformal charge-conserving deposit (Sec. 3.2) and J^3 = q alpha u^3/gamma;
 *   - the field solver of Sec. 3.3 (discrete Faraday, Ampere, auxiliary E/H,
 *     volume-weighted averages, polar-axis D^1) and the PIC loop of Sec. 3.4;
 *   - massive and massless particles (Sec. 2.3: gamma from the normalisation
 *     with m^2 = 1 or 0; massless ones are neutral);
 *   - the Wald vacuum potential (Sec. 4.1.2, eq. Wald), the BZ monopole test's
 *     initial field, particle loading, and the conserved energy / angular
 *     momentum of Sec. 2.3.
 *
 * Choices the paper leaves open are numbered readings (R1, R2, ...), named in
 * the comments where they apply and stated there.  Every function is pinned
 * by the tests in tests/test_oracle_*.py (closed forms, Table 1, conservation
 * laws, symmetry, exact reproduction of linear fields, stationarity and
 * absorption for the outer layer); the cubic shape of the absorbing ramp
 * (R16) is a reading the pins do not single out (any ramp that relaxes
 * towards the initial fields passes them).
 *
 * Layouts (shared interface, not shared code):
 *   field plane  : (n_r + 2 ng) x (n_th + 2 ng) doubles, element (i, j) at
 *                  (i + ng) * (n_th + 2 ng) + (j + ng); a component staggered to
 *                  i+1/2 (or j+1/2) is stored at index i (or j).
 *   field set    : ORC_NPLANE consecutive planes in the order of enum planes.
 *   particles    : structure of arrays, see orc_particles.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ params */

typedef struct {
  double a, M;           /* spin, mass                                   */
  double r_min, r_max;   /* radial extent, log-spaced                    */
  double dt;             /* time step (code units, r_g / c)              */
  double small_angle;    /* SMALL_ANGLE_GR clamp of theta (Sec. 3.3.2)   */
  double charge_scale;   /* deposited charge per unit weight (R13)       */
  int32_t n_r, n_th, ng; /* cells in r, theta; ghost cells per side      */
  int32_t n_iter;        /* implicit iterations (Sec. 3.1)               */
  int32_t n_filter;      /* current filter passes n_f                    */
  int32_t n_absorb;      /* outer absorbing layer cells (R16)            */
  double r0, h0;         /* quasi-spherical map (App. A): radial offset,  */
                         /* equatorial concentration; 0, 0 = log r, theta */
} orc_params;

enum {
  P_D = 0, P_B = 3, P_D0 = 6, P_B0 = 9, P_E = 12, P_H = 15,
  P_J = 18, P_J0 = 21, P_DI = 24, P_BI = 27, P_T = 30, ORC_NPLANE = 33
};

typedef struct {
  int64_t n;
  int32_t *i1, *i2;
  double *dx1, *dx2, *u1, *u2, *u3, *w, *phi;
  int32_t *i1p, *i2p;
  double *dx1p, *dx2p;
  uint8_t *tag;
} orc_particles;

#define TAG_LEAVING 0x80
#define TAG_SPECIES 0x03
#define TAG_MASSLESS 0x04 /* with species 3: a massless neutral particle */

/* Quasi-spherical map of App. A: xi = log(r - r0) uniform in x1 from the
 * inner edge r_min to r_max; theta(eta) = eta + 2 h0 eta (pi - 2 eta)(pi - eta)
 * / pi^2 with eta = x2 deta uniform on [0, pi] (reading R23: the coefficient
 * of the printed d theta / d eta is 12 h0). */
static double g_dxi(const orc_params* p)
{
  return log((p->r_max - p->r0) / (p->r_min - p->r0)) / p->n_r;
}
static double g_dth(const orc_params* p) { return M_PI / p->n_th; } /* d eta */

/* r(x1) and R = dr/dx1 = dxi (r - r0) */
static void map_r(const orc_params* p, double x1, double* r, double* R)
{
  const double dxi = g_dxi(p);
  const double e = exp(log(p->r_min - p->r0) + x1 * dxi);
  *r = p->r0 + e;
  *R = dxi * e;
}

/* theta(x2), T = d theta / d x2 and dT = d T / d x2.  Beyond either axis
 * (ghost cells) the map is continued by reflection, theta(-x2) = -theta(x2)
 * and theta(2 n_th - x2) = 2 pi - theta(x2) (reading R23: the cubic is not
 * odd about the axis for h0 != 0, and the ghost geometry must mirror the
 * interior for the axis parities of the field ghosts to hold). */
static void map_th(const orc_params* p, double x2, double* th, double* T, double* dT)
{
  double sg = 1.0, off = 0.0;
  if (x2 < 0.0) { x2 = -x2; sg = -1.0; }
  else if (x2 > p->n_th) { x2 = 2.0 * p->n_th - x2; sg = -1.0; off = 2.0 * M_PI; }
  const double de = g_dth(p), eta = x2 * de, h0 = p->h0, y = eta / M_PI;
  *th = off + sg * (eta + 2.0 * h0 * eta * (M_PI - 2.0 * eta) * (M_PI - eta) / (M_PI * M_PI));
  *T = de * (1.0 + 2.0 * h0 + 12.0 * h0 * y * (y - 1.0));
  *dT = sg * de * de * 12.0 * h0 * (2.0 * y - 1.0) / M_PI;
}

/* x2 of a polar angle: the map is linear for h0 = 0 and increasing for
 * -1/2 < h0 < 1; bisection on [0, n_th] otherwise */
static double x2_of_theta(const orc_params* p, double th)
{
  if (p->h0 == 0.0) return th / g_dth(p);
  double lo = 0.0, hi = p->n_th;
  for (int it = 0; it < 100; ++it) {
    double mid = 0.5 * (lo + hi), t, T, dT;
    map_th(p, mid, &t, &T, &dT);
    if (t < th) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* x1 of a radius */
static double x1_of_r(const orc_params* p, double r)
{
  return (log(r - p->r0) - log(p->r_min - p->r0)) / g_dxi(p);
}
static int64_t g_ld(const orc_params* p) { return (int64_t)p->n_th + 2 * p->ng; }
static int64_t g_plane(const orc_params* p) { return ((int64_t)p->n_r + 2 * p->ng) * g_ld(p); }
static int64_t IX(const orc_params* p, int i, int j)
{
  return (int64_t)(i + p->ng) * g_ld(p) + (j + p->ng);
}

int64_t orc_plane_size(const orc_params* p) { return g_plane(p); }

/* OpenMP threads the particle loop of orc_push uses */
int orc_num_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* thread count of the following parallel regions (timing of the oracle only) */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* charge-to-mass ratio per species tag (R12): e+ = +1, e- = -1, neutral = 0 */
static double tag_qm(uint8_t t)
{
  int s = t & TAG_SPECIES;
  return s == 1 ? 1.0 : (s == 2 ? -1.0 : 0.0);
}

/* ------------------------------------------------------------------ metric */

typedef struct {
  double r, th, s, c, R;          /* R = dr/dx1 = dxi (r - r0)                */
  double T, dT;                   /* T = d theta/dx2, dT = dT/dx2              */
  double Sig, Del, A, S2;         /* Sigma, Delta, A, Sigma + 2 M r            */
  double alpha, beta1;            /* lapse; contravariant shift, code units    */
  double hu11, hu22, hu33, hu13;  /* h^ij, code units                          */
  double hl11, hl22, hl33, hl13;  /* h_ij, code units                          */
  double sqrt_h, sqrt_ht;         /* sqrt(h) and sqrt(h)/sin(theta)            */
  /* first derivatives d/dx1 [0] and d/dx2 [1] of the pusher's coefficients */
  double d_alpha[2], d_beta1[2], d_hu11[2], d_hu22[2], d_hu33[2], d_hu13[2];
} orc_metric;

/*
 * Metric at code position (x1, x2) of the quasi-spherical map (App. A):
 * r = r0 + exp(xi), theta = theta(eta).  With clamp != 0, theta is clamped to
 * [small_angle, pi - small_angle] (Sec. 3.3.2, reading R4); the map's
 * derivatives are those at x2.
 *
 * Physical Kerr-Schild 3+1 quantities (App. A):
 *   Sigma = r^2 + a^2 cos^2, Delta = r^2 - 2Mr + a^2,
 *   A = (r^2+a^2)^2 - a^2 Delta sin^2, z = 2Mr/Sigma,
 *   alpha^2 = 1/(1+z), beta^r = z/(1+z),
 *   h^rr = A/(Sigma (Sigma + 2Mr)), h^rphi = a/Sigma, h^thth = 1/Sigma,
 *   h^phiphi = 1/(Sigma sin^2),
 *   h_rr = 1+z, h_rphi = -a (1+z) sin^2, h_thth = Sigma, h_phiphi = A sin^2/Sigma,
 *   sqrt(h) = Sigma sin / alpha.
 * Code components: one lower index 1 carries a factor R = dr/dx1, index 2 a
 * factor T = dtheta/dx2, index 3 a factor dphi = 1.  M enters only through
 * 2Mr (R1).  Derivatives: chain rule d/dx1 = R d/dr (dR/dx1 = dxi R),
 * d/dx2 = T d/dtheta, plus the derivative of the factor T^-2 of h^22, which
 * the printed App. A forms omit (reading R23; it vanishes for h0 = 0).
 */
void orc_metric_at(const orc_params* p, double x1, double x2, int clamp, orc_metric* m)
{
  const double a = p->a, M = p->M, dxi = g_dxi(p);
  double r, R, th, T, dT;
  map_r(p, x1, &r, &R);
  map_th(p, x2, &th, &T, &dT);
  if (clamp) {
    if (th < p->small_angle) th = p->small_angle;
    if (th > M_PI - p->small_angle) th = M_PI - p->small_angle;
  }
  double s = sin(th), c = cos(th);
  double Sig = r * r + a * a * c * c;
  double Del = r * r - 2.0 * M * r + a * a;
  double A = (r * r + a * a) * (r * r + a * a) - a * a * Del * s * s;
  double S2 = Sig + 2.0 * M * r;
  double z = 2.0 * M * r / Sig;
  double alpha = sqrt(Sig / S2);

  m->r = r; m->th = th; m->s = s; m->c = c; m->R = R; m->T = T; m->dT = dT;
  m->Sig = Sig; m->Del = Del; m->A = A; m->S2 = S2;
  m->alpha = alpha;

  double beta_r = 2.0 * M * r / S2;
  double hrr = A / (Sig * S2);
  double hrp = a / Sig;
  double htt = 1.0 / Sig;
  double hpp = 1.0 / (Sig * s * s);

  m->beta1 = beta_r / R;
  m->hu11 = hrr / (R * R);
  m->hu13 = hrp / R;
  m->hu22 = htt / (T * T);
  m->hu33 = hpp;

  m->hl11 = (1.0 + z) * R * R;
  m->hl13 = -a * (1.0 + z) * s * s * R;
  m->hl22 = Sig * T * T;
  m->hl33 = A * s * s / Sig;
  m->sqrt_ht = R * T * Sig / alpha;
  m->sqrt_h = m->sqrt_ht * s;

  /* physical derivatives */
  double dSig_r = 2.0 * r, dSig_t = -2.0 * a * a * s * c;
  double dDel_r = 2.0 * r - 2.0 * M;
  double dA_r = 4.0 * r * (r * r + a * a) - a * a * s * s * dDel_r;
  double dA_t = -2.0 * a * a * Del * s * c;
  double dS2_r = dSig_r + 2.0 * M, dS2_t = dSig_t;

  /* alpha^2 = Sig/S2 */
  double dal_r = (dSig_r * S2 - Sig * dS2_r) / (2.0 * alpha * S2 * S2);
  double dal_t = (dSig_t * S2 - Sig * dS2_t) / (2.0 * alpha * S2 * S2);
  /* beta^r = 2Mr/S2 */
  double dbr_r = (2.0 * M * S2 - 2.0 * M * r * dS2_r) / (S2 * S2);
  double dbr_t = -2.0 * M * r * dS2_t / (S2 * S2);
  /* h^rr = A/(Sig S2) */
  double den = Sig * S2;
  double dhrr_r = (dA_r * den - A * (dSig_r * S2 + Sig * dS2_r)) / (den * den);
  double dhrr_t = (dA_t * den - A * (dSig_t * S2 + Sig * dS2_t)) / (den * den);
  /* h^rphi = a/Sig, h^thth = 1/Sig */
  double dhrp_r = -a * dSig_r / (Sig * Sig), dhrp_t = -a * dSig_t / (Sig * Sig);
  double dhtt_r = -dSig_r / (Sig * Sig), dhtt_t = -dSig_t / (Sig * Sig);
  /* h^phiphi = 1/(Sig s^2) */
  double dhpp_r = -dSig_r / (Sig * Sig * s * s);
  double dhpp_t = -(dSig_t + 2.0 * Sig * c / s) / (Sig * Sig * s * s);

  /* code-coordinate derivatives */
  m->d_alpha[0] = R * dal_r;
  m->d_alpha[1] = T * dal_t;
  m->d_beta1[0] = (R * dbr_r - dxi * beta_r) / R;
  m->d_beta1[1] = T * dbr_t / R;
  m->d_hu11[0] = (R * dhrr_r - 2.0 * dxi * hrr) / (R * R);
  m->d_hu11[1] = T * dhrr_t / (R * R);
  m->d_hu13[0] = (R * dhrp_r - dxi * hrp) / R;
  m->d_hu13[1] = T * dhrp_t / R;
  m->d_hu22[0] = R * dhtt_r / (T * T);
  m->d_hu22[1] = T * dhtt_t / (T * T) - 2.0 * dT * htt / (T * T * T);
  m->d_hu33[0] = R * dhpp_r;
  m->d_hu33[1] = T * dhpp_t;
}

/* gamma = sqrt(m^2 + h^ij u_i u_j) (Sec. 2.3): m2 = 1 for massive particles,
 * 0 for massless ones */
static double gamma_m(const orc_metric* m, const double u[3], double m2)
{
  return sqrt(m2 + m->hu11 * u[0] * u[0] + m->hu22 * u[1] * u[1] + m->hu33 * u[2] * u[2] +
              2.0 * m->hu13 * u[0] * u[2]);
}

static double gamma_of(const orc_metric* m, const double u[3]) { return gamma_m(m, u, 1.0); }

/* m^2 of a slot: 0 for a neutral particle with the massless bit, else 1 */
static double tag_mass2(uint8_t t)
{
  return (t & (TAG_SPECIES | TAG_MASSLESS)) == (TAG_SPECIES | TAG_MASSLESS) ? 0.0 : 1.0;
}

/* --------------------------------------------------------------- tetrads */
/* Transforms built from the App. A matrices e^i_hat, e_i^hat (reading R22:
 * the explicit inverse rows printed beside them drop a square root).        */

/* covariant a_i -> tetrad a_hat */
void orc_cov_to_hat(const orc_metric* m, const double a[3], double ah[3])
{
  double s11 = sqrt(m->hu11);
  ah[0] = s11 * a[0] - s11 * (m->hl13 / m->hl33) * a[2];
  ah[1] = a[1] / sqrt(m->hl22);
  ah[2] = a[2] / sqrt(m->hl33);
}

/* tetrad a_hat -> covariant a_i */
void orc_hat_to_cov(const orc_metric* m, const double ah[3], double a[3])
{
  double s33 = sqrt(m->hl33);
  a[0] = ah[0] / sqrt(m->hu11) + (m->hl13 / s33) * ah[2];
  a[1] = sqrt(m->hl22) * ah[1];
  a[2] = s33 * ah[2];
}

/* contravariant A^i -> tetrad A^hat */
void orc_con_to_hat(const orc_metric* m, const double A[3], double Ah[3])
{
  double s33 = sqrt(m->hl33);
  Ah[0] = A[0] / sqrt(m->hu11);
  Ah[1] = sqrt(m->hl22) * A[1];
  Ah[2] = (m->hl13 / s33) * A[0] + s33 * A[2];
}

/* tetrad A^hat -> contravariant A^i */
void orc_hat_to_con(const orc_metric* m, const double Ah[3], double A[3])
{
  double s11 = sqrt(m->hu11);
  A[0] = s11 * Ah[0];
  A[1] = Ah[1] / sqrt(m->hl22);
  A[2] = Ah[2] / sqrt(m->hl33) - (m->hl13 / m->hl33) * s11 * Ah[0];
}

/* --------------------------------------------------------------- gather */

/* Bilinear (first-order) interpolation in code coordinates of a component
 * staggered by (o1, o2) in {0, 1/2} (reading R2).  o = 1 means a half-cell
 * offset.  Uses one ghost layer on each side. */
static double interp(const orc_params* p, const double* F, int i1, double dx1, int i2,
                     double dx2, int o1, int o2)
{
  int k1 = i1, k2 = i2;
  double w1 = dx1, w2 = dx2;
  if (o1) {
    if (dx1 >= 0.5) { w1 = dx1 - 0.5; } else { k1 = i1 - 1; w1 = dx1 + 0.5; }
  }
  if (o2) {
    if (dx2 >= 0.5) { w2 = dx2 - 0.5; } else { k2 = i2 - 1; w2 = dx2 + 0.5; }
  }
  return (1.0 - w1) * (1.0 - w2) * F[IX(p, k1, k2)] + w1 * (1.0 - w2) * F[IX(p, k1 + 1, k2)] +
         (1.0 - w1) * w2 * F[IX(p, k1, k2 + 1)] + w1 * w2 * F[IX(p, k1 + 1, k2 + 1)];
}

/* Yee locations (Sec. 3.3.1): D^1 (i+1/2, j), D^2 (i, j+1/2), D^3 (i, j),
 * B^1 (i, j+1/2), B^2 (i+1/2, j), B^3 (i+1/2, j+1/2). */
static const int STAG_D[3][2] = {{1, 0}, {0, 1}, {0, 0}};
static const int STAG_B[3][2] = {{0, 1}, {1, 0}, {1, 1}};

static void gather(const orc_params* p, const double* Dp, const double* Bp, int i1, double dx1,
                   int i2, double dx2, double D[3], double B[3])
{
  int64_t pl = g_plane(p);
  for (int k = 0; k < 3; ++k) {
    D[k] = interp(p, Dp + k * pl, i1, dx1, i2, dx2, STAG_D[k][0], STAG_D[k][1]);
    B[k] = interp(p, Bp + k * pl, i1, dx1, i2, dx2, STAG_B[k][0], STAG_B[k][1]);
  }
}

/* ----------------------------------------------------------------- Boris */

/* Textbook relativistic Boris step (Boris 1970) over a duration tau for
 * du/dt = qm (E + u x B / gamma), u the spatial 4-velocity in an orthonormal,
 * right-handed frame (Sec. 3.1, reading R10). */
void orc_boris(double u[3], const double E[3], const double B[3], double qm, double tau)
{
  double k = 0.5 * qm * tau;
  double um[3], t[3], sv[3], up[3];
  for (int c = 0; c < 3; ++c) um[c] = u[c] + k * E[c];
  double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  for (int c = 0; c < 3; ++c) t[c] = k * B[c] / g;
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int c = 0; c < 3; ++c) sv[c] = 2.0 * t[c] / (1.0 + t2);
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  double uq[3];
  uq[0] = um[0] + (up[1] * sv[2] - up[2] * sv[1]);
  uq[1] = um[1] + (up[2] * sv[0] - up[0] * sv[2]);
  uq[2] = um[2] + (up[0] * sv[1] - up[1] * sv[0]);
  for (int c = 0; c < 3; ++c) u[c] = uq[c] + k * E[c];
}

/* EM half push of Sec. 3.1 steps 3-5 (and 7-9): covariant u -> tetrad, Boris
 * for dt/2 with the FIDO-frame fields scaled by the lapse (the Lorentz term of
 * eq. equation-of-motion carries a factor alpha), back to covariant. */
static void em_half(const orc_metric* m, const double Dh[3], const double Bh[3], double qm,
                    double dt, double u[3])
{
  double E[3], B[3], uh[3];
  for (int c = 0; c < 3; ++c) { E[c] = m->alpha * Dh[c]; B[c] = m->alpha * Bh[c]; }
  orc_cov_to_hat(m, u, uh);
  orc_boris(uh, E, B, qm, 0.5 * dt);
  orc_hat_to_cov(m, uh, u);
}

/* Implicit-midpoint geodesic momentum update at fixed x^n, eq.
 * discretized-geodesic-u: n_iter fixed-point iterations on u_1, u_2; u_3 is
 * left unchanged.  The derivatives are of the contravariant h^ij (reading R5). */
static void geodesic_momentum(const orc_params* p, const orc_metric* m, double u[3], double m2)
{
  const double us1 = u[0], us2 = u[1], u3 = u[2];
  double ut1 = us1, ut2 = us2;
  for (int it = 0; it < p->n_iter; ++it) {
    double ub1 = 0.5 * (us1 + ut1), ub2 = 0.5 * (us2 + ut2);
    double ub[3] = {ub1, ub2, u3};
    double gb = gamma_m(m, ub, m2);
    double f[2];
    for (int i = 0; i < 2; ++i) {
      double quad = m->d_hu11[i] * ub1 * ub1 + m->d_hu22[i] * ub2 * ub2 +
                    m->d_hu33[i] * u3 * u3 + 2.0 * m->d_hu13[i] * ub1 * u3;
      f[i] = -gb * m->d_alpha[i] + ub1 * m->d_beta1[i] - m->alpha / (2.0 * gb) * quad;
    }
    ut1 = us1 + p->dt * f[0];
    ut2 = us2 + p->dt * f[1];
  }
  u[0] = ut1;
  u[1] = ut2;
}

/* coordinate velocity dx^i/dt = alpha h^ij u_j / gamma - beta^i (eq.
 * equation-of-motion) and dphi/dt = alpha h^3j u_j / gamma */
static void coord_velocity(const orc_metric* m, const double u[3], double v[3], double m2)
{
  double g = gamma_m(m, u, m2);
  double iu0 = m->alpha / g;
  v[0] = (m->hu11 * u[0] + m->hu13 * u[2]) * iu0 - m->beta1;
  v[1] = m->hu22 * u[1] * iu0;
  v[2] = (m->hu13 * u[0] + m->hu33 * u[2]) * iu0;
}

/* (i, dx) renormalisation after a displacement: dx in [0, 1) */
static void renorm(int32_t* i, double* dx)
{
  double f = floor(*dx);
  *i += (int32_t)f;
  *dx -= f;
  if (*dx >= 1.0) { *dx -= 1.0; *i += 1; }
}

/* One particle update, Sec. 3.1 steps 1-11, plus the particle boundaries of
 * Sec. 3.3.3.  Fields: D^n from plane P_D, B^n from plane P_B0 (left there by
 * the pre-push field stage, or the initial field). */
static void push_one(const orc_params* p, const double* F, orc_particles* P, int64_t k)
{
  uint8_t t = P->tag[k];
  if (t == 0) return;
  if (t & TAG_LEAVING) { P->tag[k] = 0; return; } /* deposited last step (R27) */
  const double qm = tag_qm(t), m2 = tag_mass2(t), dt = p->dt;
  const int64_t pl = g_plane(p);
  int32_t i1 = P->i1[k], i2 = P->i2[k];
  double dx1 = P->dx1[k], dx2 = P->dx2[k];
  double u[3] = {P->u1[k], P->u2[k], P->u3[k]};

  /* 1. previous position */
  P->i1p[k] = i1; P->i2p[k] = i2; P->dx1p[k] = dx1; P->dx2p[k] = dx2;

  const double x1 = (double)i1 + dx1, x2 = (double)i2 + dx2;
  orc_metric m;
  orc_metric_at(p, x1, x2, 1, &m);

  /* 2-9: interpolate, EM half, geodesic momentum, EM half */
  if (qm != 0.0) {
    double Dc[3], Bc[3], Dh[3], Bh[3];
    gather(p, F + P_D * pl, F + P_B0 * pl, i1, dx1, i2, dx2, Dc, Bc);
    orc_con_to_hat(&m, Dc, Dh);
    orc_con_to_hat(&m, Bc, Bh);
    em_half(&m, Dh, Bh, qm, dt, u);
    geodesic_momentum(p, &m, u, 1.0);
    em_half(&m, Dh, Bh, qm, dt, u);
  } else {
    geodesic_momentum(p, &m, u, m2); /* EM stage skipped for q = 0 */
  }

  /* 10. implicit coordinate update, eq. discretized-geodesic-x (R6, R7) */
  double d1 = 0.0, d2 = 0.0;
  for (int it = 0; it < p->n_iter; ++it) {
    orc_metric mb;
    orc_metric_at(p, x1 + 0.5 * d1, x2 + 0.5 * d2, 1, &mb);
    double v[3];
    coord_velocity(&mb, u, v, m2);
    d1 = dt * v[0];
    d2 = dt * v[1];
  }
  /* 11. out-of-plane angle at the path midpoint (R8) */
  {
    orc_metric mm;
    orc_metric_at(p, x1 + 0.5 * d1, x2 + 0.5 * d2, 1, &mm);
    double v[3];
    coord_velocity(&mm, u, v, m2);
    P->phi[k] += dt * v[2];
  }
  dx1 += d1; renorm(&i1, &dx1);
  dx2 += d2; renorm(&i2, &dx2);

  /* particle boundaries (Sec. 3.3.3): axis reflection, removal (R27) */
  if (i2 < 0) { i2 = 0; dx2 = 1.0 - dx2; u[1] = -u[1]; }
  else if (i2 >= p->n_th) { i2 = p->n_th - 1; dx2 = 1.0 - dx2; u[1] = -u[1]; }
  if (i1 < 0 || i1 >= p->n_r) t |= TAG_LEAVING;

  P->i1[k] = i1; P->i2[k] = i2; P->dx1[k] = dx1; P->dx2[k] = dx2;
  P->u1[k] = u[0]; P->u2[k] = u[1]; P->u3[k] = u[2];
  P->tag[k] = t;
}

void orc_push(const orc_params* p, const double* F, orc_particles* P)
{
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < P->n; ++k) push_one(p, F, P, k);
}

/* -------------------------------------------------------------- deposit */

/* Mirror factor of a contribution that lands on node row j (Sec. 3.3.2 with
 * reading R29): the image of a particle in the nearer polar axis deposits the
 * same contribution on an axis row (j = 0 or j = n_th) with the component's
 * axis parity, so the axis rows hold the two-sided (mirrored) values: an even
 * quantity (J^1, the charge) doubles there, the odd J^3 cancels.  Rows off
 * the axes receive nothing from the image (it lies beyond the axis). */
static double axis_image(const orc_params* p, int j, double parity)
{
  return (j == 0 || j == p->n_th) ? 1.0 + parity : 1.0;
}

/* Conformal charge-conserving deposit (Sec. 3.2, eq. charge-conservation-disc)
 * by the zigzag scheme of Umeda et al. (2003) with the first-order shape in
 * code coordinates (reading R9), from the stored previous position to the
 * stored new one (after axis reflection, R28).  J^1 at (i+1/2, j), J^2 at
 * (i, j+1/2); the out-of-plane J^3 = q (alpha/gamma) u^3 at nodes, weighted by
 * the shape at the path midpoint with theta clamped (Sec. 3.3.2, reading R11).
 * Node rows on the axes take the particle's mirror image too (axis_image).
 * Adds into planes P_J; processes particles in index order. */
static void deposit_one(const orc_params* p, double* F, const orc_particles* P, int64_t k)
{
  uint8_t t = P->tag[k];
  if (t == 0) return;
  int s = t & TAG_SPECIES;
  double sign = s == 1 ? 1.0 : (s == 2 ? -1.0 : 0.0);
  if (sign == 0.0) return;
  const double q = sign * p->charge_scale * P->w[k];
  const double dt = p->dt;
  const int64_t pl = g_plane(p);
  double* J1 = F + (P_J + 0) * pl;
  double* J2 = F + (P_J + 1) * pl;
  double* J3 = F + (P_J + 2) * pl;

  const int ia = P->i1p[k], ja = P->i2p[k];
  const int ib = P->i1[k], jb = P->i2[k];
  /* positions in the frame of the previous cell corner */
  const double xa = P->dx1p[k], ya = P->dx2p[k];
  const double xb = (double)(ib - ia) + P->dx1[k];
  const double yb = (double)(jb - ja) + P->dx2[k];
  const int ibl = ib - ia, jbl = jb - ja;

  double xr = fmin(fmin(0.0, (double)ibl) + 1.0, fmax(fmax(0.0, (double)ibl), 0.5 * (xa + xb)));
  double yr = fmin(fmin(0.0, (double)jbl) + 1.0, fmax(fmax(0.0, (double)jbl), 0.5 * (ya + yb)));

  double Fx1 = q * (xr - xa) / dt, Fy1 = q * (yr - ya) / dt;
  double Fx2 = q * (xb - xr) / dt, Fy2 = q * (yb - yr) / dt;
  double Wx1 = 0.5 * (xa + xr), Wy1 = 0.5 * (ya + yr);
  double Wx2 = 0.5 * (xr + xb) - ibl, Wy2 = 0.5 * (yr + yb) - jbl;

  J1[IX(p, ia, ja)] += Fx1 * (1.0 - Wy1) * axis_image(p, ja, 1.0);
  J1[IX(p, ia, ja + 1)] += Fx1 * Wy1 * axis_image(p, ja + 1, 1.0);
  J2[IX(p, ia, ja)] += Fy1 * (1.0 - Wx1);
  J2[IX(p, ia + 1, ja)] += Fy1 * Wx1;
  J1[IX(p, ib, jb)] += Fx2 * (1.0 - Wy2) * axis_image(p, jb, 1.0);
  J1[IX(p, ib, jb + 1)] += Fx2 * Wy2 * axis_image(p, jb + 1, 1.0);
  J2[IX(p, ib, jb)] += Fy2 * (1.0 - Wx2);
  J2[IX(p, ib + 1, jb)] += Fy2 * Wx2;

  /* out-of-plane current at the midpoint */
  double xm = 0.5 * (xa + xb), ym = 0.5 * (ya + yb);
  orc_metric m;
  orc_metric_at(p, (double)ia + xm, (double)ja + ym, 1, &m);
  double u[3] = {P->u1[k], P->u2[k], P->u3[k]};
  double v[3];
  coord_velocity(&m, u, v, 1.0); /* only charged (massive) particles deposit */
  double fm = floor(xm), gm = floor(ym);
  int km = ia + (int)fm, lm = ja + (int)gm;
  double w1 = xm - fm, w2 = ym - gm;
  double c3 = q * v[2];
  double e0 = axis_image(p, lm, -1.0), e1 = axis_image(p, lm + 1, -1.0);
  J3[IX(p, km, lm)] += c3 * (1.0 - w1) * (1.0 - w2) * e0;
  J3[IX(p, km + 1, lm)] += c3 * w1 * (1.0 - w2) * e0;
  J3[IX(p, km, lm + 1)] += c3 * (1.0 - w1) * w2 * e1;
  J3[IX(p, km + 1, lm + 1)] += c3 * w1 * w2 * e1;
}

void orc_deposit(const orc_params* p, double* F, const orc_particles* P)
{
  for (int64_t k = 0; k < P->n; ++k) deposit_one(p, F, P, k);
}

/* conformal charge sqrt(h) rho = sum q S(x - x_p) at nodes (Sec. 3.2), first-order
 * shape at the current positions, the axis rows two-sided like the deposited
 * current (axis_image); written to plane `out` (zeroed first) */
void orc_charge(const orc_params* p, const orc_particles* P, double* out)
{
  memset(out, 0, sizeof(double) * g_plane(p));
  for (int64_t k = 0; k < P->n; ++k) {
    uint8_t t = P->tag[k];
    if (t == 0) continue;
    int s = t & TAG_SPECIES;
    double sign = s == 1 ? 1.0 : (s == 2 ? -1.0 : 0.0);
    if (sign == 0.0) continue;
    double q = sign * p->charge_scale * P->w[k];
    int i = P->i1[k], j = P->i2[k];
    double w1 = P->dx1[k], w2 = P->dx2[k];
    double e0 = axis_image(p, j, 1.0), e1 = axis_image(p, j + 1, 1.0);
    out[IX(p, i, j)] += q * (1.0 - w1) * (1.0 - w2) * e0;
    out[IX(p, i + 1, j)] += q * w1 * (1.0 - w2) * e0;
    out[IX(p, i, j + 1)] += q * (1.0 - w1) * w2 * e1;
    out[IX(p, i + 1, j + 1)] += q * w1 * w2 * e1;
  }
}

/* ---------------------------------------------------------- Wald field */

/* Wald vacuum potential (Sec. 4.1.2, eq. Wald) in physical KS components,
 * A_mu = (B0/2)(g_mu3 + 2 a g_mu0):
 *   A_0 = (B0 a/2) (z (1 + cos^2) - 2)
 *   A_r = (B0 a/2) (2 z - (1 + z) sin^2)
 *   A_3 = (B0/2) sin^2 (A/Sigma - 2 a^2 z)
 * and the partial derivatives needed for E_i = d_i A_0 and B^i. */
typedef struct {
  double A0, Ar, A3;
  double dA0_r, dA0_t, dA3_r, dA3_t, dAr_t;
} orc_wald;

static void wald_at(const orc_params* p, double r, double th, double B0, orc_wald* w)
{
  const double a = p->a, M = p->M;
  double s = sin(th), c = cos(th);
  double Sig = r * r + a * a * c * c;
  double Del = r * r - 2.0 * M * r + a * a;
  double A = (r * r + a * a) * (r * r + a * a) - a * a * Del * s * s;
  double z = 2.0 * M * r / Sig;
  double dSig_r = 2.0 * r, dSig_t = -2.0 * a * a * s * c;
  double dDel_r = 2.0 * r - 2.0 * M;
  double dA_r = 4.0 * r * (r * r + a * a) - a * a * s * s * dDel_r;
  double dA_t = -2.0 * a * a * Del * s * c;
  double dz_r = 2.0 * M * (Sig - r * dSig_r) / (Sig * Sig);
  double dz_t = -2.0 * M * r * dSig_t / (Sig * Sig);

  w->A0 = 0.5 * B0 * a * (z * (1.0 + c * c) - 2.0);
  w->dA0_r = 0.5 * B0 * a * dz_r * (1.0 + c * c);
  w->dA0_t = 0.5 * B0 * a * (dz_t * (1.0 + c * c) - 2.0 * z * s * c);

  w->Ar = 0.5 * B0 * a * (2.0 * z - (1.0 + z) * s * s);
  w->dAr_t = 0.5 * B0 * a * (2.0 * dz_t - dz_t * s * s - (1.0 + z) * 2.0 * s * c);

  double Q = A / Sig - 2.0 * a * a * z;
  double dQ_r = dA_r / Sig - A * dSig_r / (Sig * Sig) - 2.0 * a * a * dz_r;
  double dQ_t = dA_t / Sig - A * dSig_t / (Sig * Sig) - 2.0 * a * a * dz_t;
  w->A3 = 0.5 * B0 * s * s * Q;
  w->dA3_r = 0.5 * B0 * s * s * dQ_r;
  w->dA3_t = 0.5 * B0 * (2.0 * s * c * Q + s * s * dQ_t);
}

/* Wald potential in code components at a code position: A_0, A_1 = R A_r, A_3 */
void orc_wald_potential(const orc_params* p, double x1, double x2, double B0, double out[3])
{
  double r, R, th, T, dT;
  map_r(p, x1, &r, &R);
  map_th(p, x2, &th, &T, &dT);
  orc_wald w;
  wald_at(p, r, th, B0, &w);
  out[0] = w.A0;
  out[1] = w.Ar * R;
  out[2] = w.A3;
}

/* analytic fields of the Wald solution at a code position (no clamp):
 * B^i = eps^ijk d_j A_k / sqrt(h) (eq. EB-set), E_i = d_i A_0, and
 * D^j = h^ji (E_i - e_ikl beta^k B^l) / alpha from eq. aux inverted (R17). */
void orc_wald_fields(const orc_params* p, double x1, double x2, double B0, double D[3],
                     double B[3])
{
  orc_metric m;
  orc_metric_at(p, x1, x2, 0, &m);
  orc_wald w;
  wald_at(p, m.r, m.th, B0, &w);
  double T = m.T, R = m.R;
  /* code derivatives: d1 = R d/dr, d2 = T d/dtheta; A_1(code) = R A_r */
  double d2A3 = T * w.dA3_t, d1A3 = R * w.dA3_r, d2A1 = T * R * w.dAr_t;
  B[0] = d2A3 / m.sqrt_h;
  B[1] = -d1A3 / m.sqrt_h;
  B[2] = -d2A1 / m.sqrt_h;
  double E1 = R * w.dA0_r, E2 = T * w.dA0_t, E3 = 0.0;
  /* sqrt(h) B^k taken from the curl directly, finite on the axis */
  double X1 = E1;
  double X2 = E2 - m.beta1 * d2A1;
  double X3 = E3 + m.beta1 * d1A3;
  D[0] = (m.hu11 * X1 + m.hu13 * X3) / m.alpha;
  D[1] = m.hu22 * X2 / m.alpha;
  D[2] = (m.hu13 * X1 + m.hu33 * X3) / m.alpha;
}

/* Wald potential planes for error bounds in tests: A_1 (code) at r-edges
 * (i+1/2, j) stored at (i, j), A_3 at nodes (i, j); every stored point. */
void orc_wald_potential_planes(const orc_params* p, double B0, double* A1, double* A3)
{
  for (int i = -p->ng; i < p->n_r + p->ng; ++i)
    for (int j = -p->ng; j < p->n_th + p->ng; ++j) {
      double a[3];
      orc_wald_potential(p, i + 0.5, j, B0, a);
      A1[IX(p, i, j)] = a[1];
      orc_wald_potential(p, i, j, B0, a);
      A3[IX(p, i, j)] = a[2];
    }
}

/* sqrt(h) at every stored point of a plane staggered by (o1, o2) half cells */
void orc_sqrt_h_plane(const orc_params* p, int o1, int o2, double* out)
{
  for (int i = -p->ng; i < p->n_r + p->ng; ++i)
    for (int j = -p->ng; j < p->n_th + p->ng; ++j) {
      orc_metric m;
      orc_metric_at(p, i + 0.5 * o1, j + 0.5 * o2, 0, &m);
      out[IX(p, i, j)] = m.sqrt_h;
    }
}

/* ------------------------------------------------------ field boundaries */

/* axis reflection (Sec. 3.3.3, figure of the staggering): r-components even,
 * theta- and phi-components odd (R3); B^2 and D^3 vanish on the axis.  kind:
 * 0 = D-like triple, 1 = B-like triple, 2 = current triple (parities as D). */
static void axis_bc(const orc_params* p, double* X, int kind)
{
  const int64_t pl = g_plane(p);
  const int ng = p->ng, nth = p->n_th;
  const int (*st)[2] = kind == 1 ? STAG_B : STAG_D;
  const double par[3] = {1.0, -1.0, -1.0};
  for (int comp = 0; comp < 3; ++comp) {
    double* C = X + comp * pl;
    int half = st[comp][1];
    for (int i = -ng; i < p->n_r + ng; ++i) {
      if (!half) {
        if (kind != 2 && ((kind == 0 && comp == 2) || (kind == 1 && comp == 1))) {
          C[IX(p, i, 0)] = 0.0;
          C[IX(p, i, nth)] = 0.0;
        }
        /* node rows run 0..nth: ng ghost rows below, ng - 1 above */
        for (int g = 1; g <= ng; ++g) C[IX(p, i, -g)] = par[comp] * C[IX(p, i, g)];
        for (int g = 1; g < ng; ++g) C[IX(p, i, nth + g)] = par[comp] * C[IX(p, i, nth - g)];
      } else {
        for (int g = 1; g <= ng; ++g) {
          C[IX(p, i, -g)] = par[comp] * C[IX(p, i, g - 1)];
          C[IX(p, i, nth - 1 + g)] = par[comp] * C[IX(p, i, nth - g)];
        }
      }
    }
  }
}

/* cubic absorbing ramp (R16): 0 inside, ((x - x0)/n_absorb)^3 capped at 1.
 * The paper fixes no value of this form; the pins fix its direction (towards
 * the initial fields) and that it absorbs, not the cubic shape. */
static double match_lambda(const orc_params* p, double x)
{
  if (p->n_absorb <= 0) return 0.0;
  double x0 = (double)(p->n_r - p->n_absorb);
  if (x <= x0) return 0.0;
  double s = (x - x0) / p->n_absorb;
  if (s > 1.0) s = 1.0;
  return s * s * s;
}

/* boundaries of an updated triple (Sec. 3.3.3): constant layer inside the
 * horizon i in [-ng, n_f] <- n_f + 1; absorbing layer towards the initial
 * field (R16); axis reflection. */
static void field_bc(const orc_params* p, double* X, const double* Xinit, int kind)
{
  const int64_t pl = g_plane(p);
  const int ng = p->ng, nth = p->n_th, nf = p->n_filter;
  const int (*st)[2] = kind == 1 ? STAG_B : STAG_D;
  for (int comp = 0; comp < 3; ++comp) {
    double* C = X + comp * pl;
    const double* C0 = Xinit + comp * pl;
    for (int i = -ng; i <= nf; ++i)
      for (int j = -ng; j < nth + ng; ++j) C[IX(p, i, j)] = C[IX(p, nf + 1, j)];
    if (p->n_absorb > 0) {
      for (int i = -ng; i < p->n_r + ng; ++i) {
        double x = (double)i + 0.5 * st[comp][0];
        double lam = match_lambda(p, x);
        if (lam == 0.0) continue;
        for (int j = -ng; j < nth + ng; ++j) {
          int64_t o = IX(p, i, j);
          C[o] = C[o] - lam * (C[o] - C0[o]);
        }
      }
    }
  }
  axis_bc(p, X, kind);
}

/* ----------------------------------------------------- grid metric */

typedef struct {
  double alpha, beta1, hl11, hl22, hl33, hl13, sqrt_h, sqrt_ht;
} gpt;

/* metric at the grid location (i + o1/2, j + o2/2), theta not clamped */
static void grid_metric(const orc_params* p, int i, int j, int o1, int o2, gpt* g)
{
  orc_metric m;
  orc_metric_at(p, i + 0.5 * o1, j + 0.5 * o2, 0, &m);
  g->alpha = m.alpha; g->beta1 = m.beta1;
  g->hl11 = m.hl11; g->hl22 = m.hl22; g->hl33 = m.hl33; g->hl13 = m.hl13;
  g->sqrt_h = m.sqrt_h; g->sqrt_ht = m.sqrt_ht;
}

/* polar area A_{i+1/2} = R (r^2+a^2) sqrt(1 + 2Mr/(r^2+a^2)) (1 - cos theta_c)
 * at r(i+1/2), over the cap from the axis to theta_c = theta(x2 = 1/2)
 * (Sec. 3.3.2, App. A "Spherical Kerr-Schild", dr -> R, the cap edge through
 * the quasi-spherical map) */
static double polar_area(const orc_params* p, int i)
{
  double r, R, thc, T, dT;
  map_r(p, i + 0.5, &r, &R);
  map_th(p, 0.5, &thc, &T, &dT);
  double ra = r * r + p->a * p->a;
  return R * ra * sqrt(1.0 + 2.0 * p->M * r / ra) * (1.0 - cos(thc));
}

/* ------------------------------------------------------ aux E and H */

/* eq. discretized-auxE / -auxH: E_i from (B, D), volume-weighted radial
 * averages <.> with weights sqrt(h)/sin(theta) (Sec. 3.3.1).  Computed for
 * i in [-1, n_r] (radial index of the component's own location). */
static void aux_E(const orc_params* p, const double* Bs, const double* Ds, double* E)
{
  const int64_t pl = g_plane(p);
  const double *D1 = Ds, *D3 = Ds + 2 * pl, *D2 = Ds + pl;
  const double *B2 = Bs + pl, *B3 = Bs + 2 * pl;
  double *E1 = E, *E2 = E + pl, *E3 = E + 2 * pl;
  for (int i = -1; i <= p->n_r; ++i) {
    for (int j = 0; j <= p->n_th; ++j) {
      gpt c, m0, m1;
      /* E_1 at (i+1/2, j): <h13 D3> from D3(i, j), D3(i+1, j) */
      grid_metric(p, i, j, 1, 0, &c);
      grid_metric(p, i, j, 0, 0, &m0);
      grid_metric(p, i + 1, j, 0, 0, &m1);
      double av = (m0.sqrt_ht * m0.hl13 * D3[IX(p, i, j)] +
                   m1.sqrt_ht * m1.hl13 * D3[IX(p, i + 1, j)]) / (2.0 * c.sqrt_ht);
      E1[IX(p, i, j)] = c.alpha * (c.hl11 * D1[IX(p, i, j)] + av);
      /* E_3 at (i, j): <h13 D1>, <sqrt(h) beta1 B2> from (i-1/2), (i+1/2) */
      grid_metric(p, i, j, 0, 0, &c);
      grid_metric(p, i - 1, j, 1, 0, &m0);
      grid_metric(p, i, j, 1, 0, &m1);
      double a1 = (m0.sqrt_ht * m0.hl13 * D1[IX(p, i - 1, j)] +
                   m1.sqrt_ht * m1.hl13 * D1[IX(p, i, j)]) / (2.0 * c.sqrt_ht);
      double a2 = (m0.sqrt_ht * m0.sqrt_h * m0.beta1 * B2[IX(p, i - 1, j)] +
                   m1.sqrt_ht * m1.sqrt_h * m1.beta1 * B2[IX(p, i, j)]) / (2.0 * c.sqrt_ht);
      E3[IX(p, i, j)] = c.alpha * (c.hl33 * D3[IX(p, i, j)] + a1) + a2;
      if (j < p->n_th) {
        /* E_2 at (i, j+1/2): <sqrt(h) beta1 B3> from (i-1/2, j+1/2), (i+1/2, j+1/2) */
        grid_metric(p, i, j, 0, 1, &c);
        grid_metric(p, i - 1, j, 1, 1, &m0);
        grid_metric(p, i, j, 1, 1, &m1);
        double a3 = (m0.sqrt_ht * m0.sqrt_h * m0.beta1 * B3[IX(p, i - 1, j)] +
                     m1.sqrt_ht * m1.sqrt_h * m1.beta1 * B3[IX(p, i, j)]) / (2.0 * c.sqrt_ht);
        E2[IX(p, i, j)] = c.alpha * c.hl22 * D2[IX(p, i, j)] - a3;
      }
    }
  }
}

static void aux_H(const orc_params* p, const double* Bs, const double* Ds, double* H)
{
  const int64_t pl = g_plane(p);
  const double *D2 = Ds + pl, *D3 = Ds + 2 * pl;
  const double *B1 = Bs, *B2 = Bs + pl, *B3 = Bs + 2 * pl;
  double *H1 = H, *H2 = H + pl, *H3 = H + 2 * pl;
  for (int i = -1; i <= p->n_r; ++i) {
    for (int j = 0; j <= p->n_th; ++j) {
      gpt c, m0, m1;
      /* H_2 at (i+1/2, j): <sqrt(h) beta1 D3> from D3(i, j), D3(i+1, j) */
      grid_metric(p, i, j, 1, 0, &c);
      grid_metric(p, i, j, 0, 0, &m0);
      grid_metric(p, i + 1, j, 0, 0, &m1);
      double a1 = (m0.sqrt_ht * m0.sqrt_h * m0.beta1 * D3[IX(p, i, j)] +
                   m1.sqrt_ht * m1.sqrt_h * m1.beta1 * D3[IX(p, i + 1, j)]) / (2.0 * c.sqrt_ht);
      H2[IX(p, i, j)] = c.alpha * c.hl22 * B2[IX(p, i, j)] + a1;
      if (j < p->n_th) {
        /* H_1 at (i, j+1/2): <h13 B3> from B3(i-1/2, j+1/2), B3(i+1/2, j+1/2) */
        grid_metric(p, i, j, 0, 1, &c);
        grid_metric(p, i - 1, j, 1, 1, &m0);
        grid_metric(p, i, j, 1, 1, &m1);
        double a2 = (m0.sqrt_ht * m0.hl13 * B3[IX(p, i - 1, j)] +
                     m1.sqrt_ht * m1.hl13 * B3[IX(p, i, j)]) / (2.0 * c.sqrt_ht);
        H1[IX(p, i, j)] = c.alpha * (c.hl11 * B1[IX(p, i, j)] + a2);
        /* H_3 at (i+1/2, j+1/2): <h13 B1>, <sqrt(h) beta1 D2> from (i, j+1/2), (i+1, j+1/2) */
        grid_metric(p, i, j, 1, 1, &c);
        grid_metric(p, i, j, 0, 1, &m0);
        grid_metric(p, i + 1, j, 0, 1, &m1);
        double a3 = (m0.sqrt_ht * m0.hl13 * B1[IX(p, i, j)] +
                     m1.sqrt_ht * m1.hl13 * B1[IX(p, i + 1, j)]) / (2.0 * c.sqrt_ht);
        double a4 = (m0.sqrt_ht * m0.sqrt_h * m0.beta1 * D2[IX(p, i, j)] +
                     m1.sqrt_ht * m1.sqrt_h * m1.beta1 * D2[IX(p, i + 1, j)]) / (2.0 * c.sqrt_ht);
        H3[IX(p, i, j)] = c.alpha * (c.hl33 * B3[IX(p, i, j)] + a3) - a4;
      }
    }
  }
}

/* ------------------------------------------------------ Faraday, Ampere */

/* eq. discretized-faraday: X <- X - dt curl(E)/sqrt(h) on the evolved range
 * (B^1: i in [0, n_r], j in [0, n_th); B^2: i in [0, n_r), j in [1, n_th);
 * B^3: i in [0, n_r), j in [0, n_th)); unit code spacing. */
static void faraday(const orc_params* p, double* X, const double* E, double dt)
{
  const int64_t pl = g_plane(p);
  const double *E1 = E, *E2 = E + pl, *E3 = E + 2 * pl;
  double *X1 = X, *X2 = X + pl, *X3 = X + 2 * pl;
  for (int i = 0; i <= p->n_r; ++i)
    for (int j = 0; j < p->n_th; ++j) {
      gpt g;
      grid_metric(p, i, j, 0, 1, &g);
      X1[IX(p, i, j)] -= dt * (E3[IX(p, i, j + 1)] - E3[IX(p, i, j)]) / g.sqrt_h;
    }
  for (int i = 0; i < p->n_r; ++i)
    for (int j = 1; j < p->n_th; ++j) {
      gpt g;
      grid_metric(p, i, j, 1, 0, &g);
      X2[IX(p, i, j)] += dt * (E3[IX(p, i + 1, j)] - E3[IX(p, i, j)]) / g.sqrt_h;
    }
  for (int i = 0; i < p->n_r; ++i)
    for (int j = 0; j < p->n_th; ++j) {
      gpt g;
      grid_metric(p, i, j, 1, 1, &g);
      double curl = (E2[IX(p, i + 1, j)] - E2[IX(p, i, j)]) - (E1[IX(p, i, j + 1)] - E1[IX(p, i, j)]);
      X3[IX(p, i, j)] -= dt * curl / g.sqrt_h;
    }
}

/* eq. discretized-ampere: X <- X + dt (curl H - 4 pi J)/sqrt(h) with J the
 * average of w0 * J0 + w1 * J1 (planes); D^1 on the axis rows by the integral
 * (polar-cap) form of Sec. 3.3.2 with the cap area A_{i+1/2} and the printed
 * 2 pi, which goes with the two-sided (mirrored) axis-row current the deposit
 * leaves there (R29).  At theta = pi the cap is bounded with the opposite
 * orientation (R29). */
static void ampere(const orc_params* p, double* X, const double* H, const double* Ja,
                   const double* Jb, double wa, double wb, double dt)
{
  const int64_t pl = g_plane(p);
  const double *H1 = H, *H2 = H + pl, *H3 = H + 2 * pl;
  double *X1 = X, *X2 = X + pl, *X3 = X + 2 * pl;
  const double fpi = 4.0 * M_PI, tpi = 2.0 * M_PI;
#define JJ(c, o) (wa * Ja[(c) * pl + (o)] + wb * Jb[(c) * pl + (o)])
  for (int i = 0; i < p->n_r; ++i) {
    for (int j = 1; j < p->n_th; ++j) {
      gpt g;
      grid_metric(p, i, j, 1, 0, &g);
      int64_t o = IX(p, i, j);
      X1[o] += dt * ((H3[IX(p, i, j)] - H3[IX(p, i, j - 1)]) - fpi * JJ(0, o)) / g.sqrt_h;
    }
    double Ap = polar_area(p, i);
    int64_t o0 = IX(p, i, 0), on = IX(p, i, p->n_th);
    X1[o0] += dt * (H3[IX(p, i, 0)] - tpi * JJ(0, o0)) / Ap;
    X1[on] += dt * (-H3[IX(p, i, p->n_th - 1)] - tpi * JJ(0, on)) / Ap;
  }
  for (int i = 0; i <= p->n_r; ++i)
    for (int j = 0; j < p->n_th; ++j) {
      gpt g;
      grid_metric(p, i, j, 0, 1, &g);
      int64_t o = IX(p, i, j);
      X2[o] += dt * (-(H3[IX(p, i, j)] - H3[IX(p, i - 1, j)]) - fpi * JJ(1, o)) / g.sqrt_h;
    }
  for (int i = 0; i <= p->n_r; ++i)
    for (int j = 1; j < p->n_th; ++j) {
      gpt g;
      grid_metric(p, i, j, 0, 0, &g);
      int64_t o = IX(p, i, j);
      double curl = (H2[IX(p, i, j)] - H2[IX(p, i - 1, j)]) - (H1[IX(p, i, j)] - H1[IX(p, i, j - 1)]);
      X3[o] += dt * (curl - fpi * JJ(2, o)) / g.sqrt_h;
    }
#undef JJ
}

/* ------------------------------------------------------ current filter */

/* n_f passes of the separable (1,2,1)/4 x (1,2,1)/4 binomial filter on each
 * current component (R15); theta ghosts by the axis parities before each pass;
 * applied for i in [1 - ng, n_r + ng - 2] and the physical theta range. */
static void filter_currents(const orc_params* p, double* F)
{
  const int64_t pl = g_plane(p);
  double* J = F + P_J * pl;
  double* T = F + P_T * pl;
  for (int pass = 0; pass < p->n_filter; ++pass) {
    axis_bc(p, J, 2);
    memcpy(T, J, sizeof(double) * 3 * pl);
    for (int comp = 0; comp < 3; ++comp) {
      int jmax = STAG_D[comp][1] ? p->n_th - 1 : p->n_th;
      double* C = J + comp * pl;
      const double* S = T + comp * pl;
      for (int i = 1 - p->ng; i <= p->n_r + p->ng - 2; ++i)
        for (int j = 0; j <= jmax; ++j) {
          double acc = 0.0;
          for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b) {
              double wa = a == 0 ? 0.5 : 0.25, wb = b == 0 ? 0.5 : 0.25;
              acc += wa * wb * S[IX(p, i + a, j + b)];
            }
          C[IX(p, i, j)] = acc;
        }
    }
  }
}

/* same filter on a single node-located scalar plane (even axis parity), used
 * for the filtered charge of the Gauss-law check */
static void filter_scalar(const orc_params* p, double* C, double* T)
{
  const int64_t pl = g_plane(p);
  const int ng = p->ng, nth = p->n_th;
  for (int pass = 0; pass < p->n_filter; ++pass) {
    for (int i = -ng; i < p->n_r + ng; ++i) {
      for (int g = 1; g <= ng; ++g) C[IX(p, i, -g)] = C[IX(p, i, g)];
      for (int g = 1; g < ng; ++g) C[IX(p, i, nth + g)] = C[IX(p, i, nth - g)];
    }
    memcpy(T, C, sizeof(double) * pl);
    for (int i = 1 - ng; i <= p->n_r + ng - 2; ++i)
      for (int j = 0; j <= nth; ++j) {
        double acc = 0.0;
        for (int a = -1; a <= 1; ++a)
          for (int b = -1; b <= 1; ++b) {
            double wa = a == 0 ? 0.5 : 0.25, wb = b == 0 ? 0.5 : 0.25;
            acc += wa * wb * T[IX(p, i + a, j + b)];
          }
        C[IX(p, i, j)] = acc;
      }
  }
}

/* ------------------------------------------------------ PIC loop stages */

/* Sec. 3.4, step 2 (before the push):
 *   B^{n-1} = (B^{n-3/2} + B^{n-1/2})/2 and D^{n-1/2} = (D^{n-1} + D^n)/2 in em0,
 *   E^{n-1/2} from (B^{n-1/2}, D^{n-1/2}),
 *   auxiliary Faraday B^{n-1} -> B^n in em0.
 * Sec. 3.4, steps 5-8 (after the deposit):
 *   filter J^{n+1/2}; E^n, H^n from (B^n, D^n); main Faraday em.B -> B^{n+1/2}
 *   (old B^{n-1/2} kept in em0); auxiliary Ampere D^{n-1/2} -> D^{n+1/2} with
 *   J^n = (J^{n-1/2} + J^{n+1/2})/2; H^{n+1/2} from (B^{n+1/2}, D^{n+1/2});
 *   final Ampere D^n -> D^{n+1} with J^{n+1/2} (old D^n kept in em0);
 *   cur0 <- cur, cur <- 0.
 * Boundaries after every substep on the triple it updated. */
void orc_field_advance(const orc_params* p, double* F, int stage)
{
  const int64_t pl = g_plane(p);
  double *D = F + P_D * pl, *B = F + P_B * pl, *D0 = F + P_D0 * pl, *B0 = F + P_B0 * pl;
  double *E = F + P_E * pl, *H = F + P_H * pl, *J = F + P_J * pl, *J0 = F + P_J0 * pl;
  const double *DI = F + P_DI * pl, *BI = F + P_BI * pl;
  const double dt = p->dt;
  if (stage == 0) {
    for (int64_t o = 0; o < 3 * pl; ++o) {
      B0[o] = 0.5 * (B0[o] + B[o]);
      D0[o] = 0.5 * (D0[o] + D[o]);
    }
    aux_E(p, B, D0, E);
    faraday(p, B0, E, dt);
    field_bc(p, B0, BI, 1);
  } else {
    filter_currents(p, F);
    aux_E(p, B0, D, E);
    aux_H(p, B0, D, H);
    memcpy(B0, B, sizeof(double) * 3 * pl);
    faraday(p, B, E, dt);
    field_bc(p, B, BI, 1);
    ampere(p, D0, H, J0, J, 0.5, 0.5, dt);
    field_bc(p, D0, DI, 0);
    aux_H(p, B, D0, H);
    memcpy(D0, D, sizeof(double) * 3 * pl);
    ampere(p, D, H, J, J, 1.0, 0.0, dt);
    field_bc(p, D, DI, 0);
    memcpy(J0, J, sizeof(double) * 3 * pl);
    memset(J, 0, sizeof(double) * 3 * pl);
  }
}

/* ------------------------------------------------------ Wald init */

/* Wald initial data (Sec. 4.1.2): A_3 on nodes (i, j) and A_1 on r-edges
 * (i+1/2, j); B by the discrete Stokes curl of eq. EB-set,
 *   B^1(i, j+1/2) = (A_3(i, j+1) - A_3(i, j)) / sqrt(h),
 *   B^2(i+1/2, j) = -(A_3(i+1, j) - A_3(i, j)) / sqrt(h),
 *   B^3(i+1/2, j+1/2) = -(A_1(i+1/2, j+1) - A_1(i+1/2, j)) / sqrt(h);
 * D pointwise from the analytic solution (R17).  Sets em, em0, the absorbing
 * targets, zeroes aux, cur, cur0; axis boundaries applied.  Points whose
 * stencil leaves the array (last row/column) take the analytic B. */
void orc_fields_init_wald(const orc_params* p, double* F, double B0v)
{
  const int64_t pl = g_plane(p);
  const int ng = p->ng;
  memset(F, 0, sizeof(double) * ORC_NPLANE * pl);
  double *D = F + P_D * pl, *B = F + P_B * pl;
  for (int i = -ng; i < p->n_r + ng; ++i) {
    for (int j = -ng; j < p->n_th + ng; ++j) {
      int64_t o = IX(p, i, j);
      double Dv[3], Bv[3], pa[3], pb[3];
      for (int k = 0; k < 3; ++k) {
        orc_wald_fields(p, i + 0.5 * STAG_D[k][0], j + 0.5 * STAG_D[k][1], B0v, Dv, Bv);
        D[k * pl + o] = Dv[k];
      }
      int last_i = (i == p->n_r + ng - 1), last_j = (j == p->n_th + ng - 1);
      /* B^1 (i, j+1/2) */
      if (!last_j) {
        orc_metric m; orc_metric_at(p, i, j + 0.5, 0, &m);
        orc_wald_potential(p, i, j, B0v, pa);
        orc_wald_potential(p, i, j + 1, B0v, pb);
        B[0 * pl + o] = (pb[2] - pa[2]) / m.sqrt_h;
      } else {
        orc_wald_fields(p, i, j + 0.5, B0v, Dv, Bv);
        B[0 * pl + o] = Bv[0];
      }
      /* B^2 (i+1/2, j) */
      if (!last_i) {
        orc_metric m; orc_metric_at(p, i + 0.5, j, 0, &m);
        orc_wald_potential(p, i, j, B0v, pa);
        orc_wald_potential(p, i + 1, j, B0v, pb);
        B[1 * pl + o] = -(pb[2] - pa[2]) / m.sqrt_h;
      } else {
        orc_wald_fields(p, i + 0.5, j, B0v, Dv, Bv);
        B[1 * pl + o] = Bv[1];
      }
      /* B^3 (i+1/2, j+1/2) */
      if (!last_j) {
        orc_metric m; orc_metric_at(p, i + 0.5, j + 0.5, 0, &m);
        orc_wald_potential(p, i + 0.5, j, B0v, pa);
        orc_wald_potential(p, i + 0.5, j + 1, B0v, pb);
        B[2 * pl + o] = -(pb[1] - pa[1]) / m.sqrt_h;
      } else {
        orc_wald_fields(p, i + 0.5, j + 0.5, B0v, Dv, Bv);
        B[2 * pl + o] = Bv[2];
      }
    }
  }
  axis_bc(p, D, 0);
  axis_bc(p, B, 1);
  memcpy(F + P_D0 * pl, D, sizeof(double) * 3 * pl);
  memcpy(F + P_B0 * pl, B, sizeof(double) * 3 * pl);
  memcpy(F + P_DI * pl, D, sizeof(double) * 3 * pl);
  memcpy(F + P_BI * pl, B, sizeof(double) * 3 * pl);
}

/* Monopole initial data of the BZ test (Sec. "BZ monopole", eq. for A_phi):
 * A_phi = -B0 cos(theta), so the discrete curl (eq. EB-set) gives
 * B^1 (i, j+1/2) = (A_3(j+1) - A_3(j)) / sqrt(h) and B^2 = B^3 = 0; D = 0.
 * The last ghost column has no j+1 node and takes the analytic value
 * B^1 = T B0 sin(theta) / sqrt(h), T = dtheta/dx2 (the axis pass then
 * overwrites it). */
void orc_fields_init_monopole(const orc_params* p, double* F, double B0v)
{
  const int64_t pl = g_plane(p);
  const int ng = p->ng;
  memset(F, 0, sizeof(double) * ORC_NPLANE * pl);
  double *D = F + P_D * pl, *B = F + P_B * pl;
  for (int i = -ng; i < p->n_r + ng; ++i)
    for (int j = -ng; j < p->n_th + ng; ++j) {
      orc_metric m;
      orc_metric_at(p, i, j + 0.5, 0, &m);
      if (j < p->n_th + ng - 1) {
        double ta, tb, T, dT;
        map_th(p, j, &ta, &T, &dT);
        map_th(p, j + 1, &tb, &T, &dT);
        const double a3 = -B0v * cos(ta), b3 = -B0v * cos(tb);
        B[IX(p, i, j)] = (b3 - a3) / m.sqrt_h;
      } else {
        B[IX(p, i, j)] = m.T * B0v * sin(m.th) / m.sqrt_h;
      }
    }
  axis_bc(p, D, 0);
  axis_bc(p, B, 1);
  memcpy(F + P_D0 * pl, D, sizeof(double) * 3 * pl);
  memcpy(F + P_B0 * pl, B, sizeof(double) * 3 * pl);
  memcpy(F + P_DI * pl, D, sizeof(double) * 3 * pl);
  memcpy(F + P_BI * pl, B, sizeof(double) * 3 * pl);
}

/* ------------------------------------------------------ Philox, loading */

/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
 * round multipliers 0xD2511F53, 0xCD9E8D57, Weyl key increments 0x9E3779B9,
 * 0xBB67AE85, ten rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* counter (idx, sub, stream, k): sub = 0 for the initial loading, 1 + call for
 * the injection call `call` */
static void draw_sub(uint64_t seed, uint32_t idx, uint32_t sub, uint32_t stream, uint32_t k,
                     uint32_t out[4])
{
  uint32_t ctr[4] = {idx, sub, stream, k};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

static void draw(uint64_t seed, uint32_t idx, uint32_t stream, uint32_t k, uint32_t out[4])
{
  uint32_t ctr[4] = {idx, 0u, stream, k};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

#define U01_OPEN0(w) (((double)(w) + 1.0) * 2.3283064365386963e-10) /* (0, 1] */
#define U01_HALF(w) (((double)(w) + 0.5) * 2.3283064365386963e-10)  /* (0, 1) */
#define U01_LOW(w) ((double)(w) * 2.3283064365386963e-10)           /* [0, 1) */

/* Isotropic Maxwell-Juttner sample of the spatial 4-velocity at temperature T
 * (units of m c^2) by Sobol's rejection method as given by Zenitani (2015,
 * Phys. Plasmas 22, 042116): u = -T ln(X1 X2 X3), eta = -T ln(X1 X2 X3 X4),
 * accept if eta^2 - u^2 > 1; direction from two more uniforms. */
static void mj_sample(uint64_t seed, uint32_t q, uint32_t sub, double T, double uh[3])
{
  double u = 0.0;
  for (uint32_t k = 0; k < 4096u; ++k) {
    uint32_t w[4];
    draw_sub(seed, q, sub, 1u, k, w);
    double x1 = U01_OPEN0(w[0]), x2 = U01_OPEN0(w[1]), x3 = U01_OPEN0(w[2]), x4 = U01_OPEN0(w[3]);
    u = -T * log(x1 * x2 * x3);
    double eta = -T * log(x1 * x2 * x3 * x4);
    if (eta * eta - u * u > 1.0) break;
  }
  uint32_t w[4];
  draw_sub(seed, q, sub, 2u, 0u, w);
  double x5 = U01_HALF(w[0]), x6 = U01_HALF(w[1]);
  double st = 2.0 * u * sqrt(x5 * (1.0 - x5));
  uh[0] = u * (2.0 * x5 - 1.0);
  uh[1] = st * cos(2.0 * M_PI * x6);
  uh[2] = st * sin(2.0 * M_PI * x6);
}

/*
 * Particle loading (reading R18, R19).
 * Pairs k = 0 .. n_pairs-1 occupy slots 2k (e+, tag 1) and 2k+1 (e-, tag 2) at one
 * position (zero net charge at t = 0).  With ppc > 0, pair k sits in cell
 * c = k / (ppc/2), c = i1 * n_th + i2; otherwise c is uniform over all cells.
 * Offsets dx1, dx2 uniform in [0, 1).  Each particle's momentum is an isotropic
 * Maxwell-Juttner sample in the FIDO tetrad frame, u_i = e_i^hat u_hat at the
 * particle (theta clamped).  Slots 2 n_pairs .. n-1 are n_geo neutral test
 * particles (tag 3): r in U[6, 15], theta in U[pi/3, 2pi/3], tetrad velocity
 * u_phihat = (0.9 + 0.2 X) sqrt(M/(r - 3M)), u_rhat, u_thhat in 0.05 U[-1, 1],
 * accepted when bound, E = alpha gamma - beta^1 u_1 < 1.  Random numbers:
 * Philox4x32-10, key = seed, counter = (index, 0, stream, k); streams: 0
 * position (pair index), 1 momentum attempts, 2 direction, 3/4 geodesics.
 */
void orc_particles_init(const orc_params* p, orc_particles* P, int64_t n_pairs, int32_t ppc,
                        double T, int64_t n_geo, uint64_t seed)
{
  const int64_t ncell = (int64_t)p->n_r * p->n_th;
  for (int64_t k = 0; k < n_pairs; ++k) {
    uint32_t w[4];
    draw(seed, (uint32_t)k, 0u, 0u, w);
    int64_t c;
    if (ppc > 0) c = k / (ppc / 2);
    else c = (int64_t)((((uint64_t)w[2] << 32) | w[3]) % (uint64_t)ncell);
    int32_t i1 = (int32_t)(c / p->n_th), i2 = (int32_t)(c % p->n_th);
    double dx1 = U01_LOW(w[0]), dx2 = U01_LOW(w[1]);
    orc_metric m;
    orc_metric_at(p, i1 + dx1, i2 + dx2, 1, &m);
    for (int s = 0; s < 2; ++s) {
      int64_t q = 2 * k + s;
      double uh[3], u[3];
      mj_sample(seed, (uint32_t)q, 0u, T, uh);
      orc_hat_to_cov(&m, uh, u);
      P->i1[q] = i1; P->i2[q] = i2; P->dx1[q] = dx1; P->dx2[q] = dx2;
      P->i1p[q] = i1; P->i2p[q] = i2; P->dx1p[q] = dx1; P->dx2p[q] = dx2;
      P->u1[q] = u[0]; P->u2[q] = u[1]; P->u3[q] = u[2];
      P->w[q] = 1.0; P->phi[q] = 0.0;
      P->tag[q] = (uint8_t)(s == 0 ? 1 : 2);
    }
  }
  for (int64_t g = 0; g < n_geo; ++g) {
    int64_t q = 2 * n_pairs + g;
    int32_t i1 = 0, i2 = 0;
    double dx1 = 0.0, dx2 = 0.0, u[3] = {0.0, 0.0, 0.0};
    for (uint32_t k = 0; k < 64u; ++k) {
      uint32_t w[4], v[4];
      draw(seed, (uint32_t)g, 3u, k, w);
      draw(seed, (uint32_t)g, 4u, k, v);
      double r = 6.0 + 9.0 * U01_LOW(w[0]);
      double th = M_PI / 3.0 + (M_PI / 3.0) * U01_LOW(w[1]);
      double x1 = x1_of_r(p, r), x2 = x2_of_theta(p, th);
      double f1 = floor(x1), f2 = floor(x2);
      i1 = (int32_t)f1; dx1 = x1 - f1;
      i2 = (int32_t)f2; dx2 = x2 - f2;
      orc_metric m;
      orc_metric_at(p, i1 + dx1, i2 + dx2, 1, &m);
      double uk = sqrt(p->M / (m.r - 3.0 * p->M));
      double uh[3] = {0.05 * (2.0 * U01_LOW(w[3]) - 1.0), 0.05 * (2.0 * U01_LOW(v[0]) - 1.0),
                      (0.9 + 0.2 * U01_LOW(w[2])) * uk};
      orc_hat_to_cov(&m, uh, u);
      double E = m.alpha * gamma_of(&m, u) - m.beta1 * u[0];
      if (E < 1.0) break;
    }
    P->i1[q] = i1; P->i2[q] = i2; P->dx1[q] = dx1; P->dx2[q] = dx2;
    P->i1p[q] = i1; P->i2p[q] = i2; P->dx1p[q] = dx1; P->dx2p[q] = dx2;
    P->u1[q] = u[0]; P->u2[q] = u[1]; P->u3[q] = u[2];
    P->w[q] = 1.0; P->phi[q] = 0.0;
    P->tag[q] = 3;
  }
}

/* ------------------------------------------------------ pair injection */

/*
 * Pair injection where the plasma is strongly magnetised (Sec. 4.4 and
 * Sec. 4.5: e+- pairs at temperature T are added wherever the local
 * magnetisation sigma = B_i B^i / (4 pi n m) exceeds a threshold; reading R30):
 *
 *  - sigma per cell (i, j), i in [i_lo, i_hi), j in [0, n_th), at the cell
 *    centre (i + 1/2, j + 1/2): B^1 is the mean of its two r-faces' values
 *    (stored at (i, j + 1/2) and (i + 1, j + 1/2)), B^2 the mean of its two
 *    theta-faces' ((i + 1/2, j), (i + 1/2, j + 1)), B^3 its own value; plane B
 *    of the field set;  B_i B^i = h_ij B^i B^j with the code-unit spatial
 *    metric at the centre;
 *  - n = kappa sum w / sqrt(h) over the live, not leaving e+ and e- (species
 *    1, 2, any slot) whose cell is (i, j): the number density with the normalisation
 *    of the deposited charge (sqrt(h) rho = kappa q sum w S), m = 1;
 *  - a cell injects when B_i B^i > 0 and B_i B^i >= 4 pi sigma_th n (an
 *    empty magnetised cell has sigma = infinity);
 *  - every injecting cell, in the order c = i n_th + j, adds n_inj pairs;
 *    pair k (counted over the call) fills slots first_free + 2k (e+, tag 1)
 *    and first_free + 2k + 1 (e-, tag 2) at one position (zero net charge),
 *    offsets uniform in the cell, momenta isotropic Maxwell-Juttner at T in
 *    the FIDO tetrad frame at that position, weight w_inj, phi = 0; pairs
 *    that would not fit below n are not injected;
 *  - random numbers: Philox4x32-10 with key = seed and counter
 *    (index, 1 + call, stream, k): streams 0 position (pair index k),
 *    1 momentum attempts and 2 direction (particle index 2k + s).
 * Returns the number of pairs injected.
 */
/* weight sum of the live, not leaving e+ and e- per cell (n_r x n_th) */
static double* cell_weights(const orc_params* p, const orc_particles* P)
{
  double* wsum = (double*)calloc((size_t)p->n_r * p->n_th, sizeof(double));
  for (int64_t q = 0; q < P->n; ++q) {
    uint8_t t = P->tag[q];
    int s = t & TAG_SPECIES;
    if (t == 0 || (t & TAG_LEAVING) || (s != 1 && s != 2)) continue;
    int i = P->i1[q], j = P->i2[q];
    if (i < 0 || i >= p->n_r || j < 0 || j >= p->n_th) continue;
    wsum[(int64_t)i * p->n_th + j] += P->w[q];
  }
  return wsum;
}

/* B_i B^i and the number density n at the centre of cell (i, j) */
static void cell_magnetisation(const orc_params* p, const double* F, const double* wsum, int i, int j,
                               double* bb, double* n)
{
  const int64_t pl = g_plane(p);
  const double *B1 = F + P_B * pl, *B2 = F + (P_B + 1) * pl, *B3 = F + (P_B + 2) * pl;
  orc_metric m;
  orc_metric_at(p, i + 0.5, j + 0.5, 0, &m);
  double b1 = 0.5 * (B1[IX(p, i, j)] + B1[IX(p, i + 1, j)]);
  double b2 = 0.5 * (B2[IX(p, i, j)] + B2[IX(p, i, j + 1)]);
  double b3 = B3[IX(p, i, j)];
  *bb = m.hl11 * b1 * b1 + 2.0 * m.hl13 * b1 * b3 + m.hl22 * b2 * b2 + m.hl33 * b3 * b3;
  *n = p->charge_scale * wsum[(int64_t)i * p->n_th + j] / m.sqrt_h;
}

int64_t orc_inject_pairs(const orc_params* p, const double* F, orc_particles* P, double sigma_th,
                         double T, int32_t n_inj, double w_inj, int32_t i_lo, int32_t i_hi,
                         uint64_t seed, uint32_t call, int64_t first_free)
{
  double* wsum = cell_weights(p, P);
  int64_t k = 0;
  const uint32_t sub = call + 1u;
  if (i_lo < 0) i_lo = 0;
  if (i_hi > p->n_r) i_hi = p->n_r;
  for (int i = i_lo; i < i_hi; ++i) {
    for (int j = 0; j < p->n_th; ++j) {
      double bb, n;
      cell_magnetisation(p, F, wsum, i, j, &bb, &n);
      if (!(bb > 0.0 && bb >= 4.0 * M_PI * sigma_th * n)) continue;
      for (int32_t e = 0; e < n_inj; ++e, ++k) {
        int64_t q0 = first_free + 2 * k;
        if (q0 + 1 >= P->n) { free(wsum); return k; }
        uint32_t w[4];
        draw_sub(seed, (uint32_t)k, sub, 0u, 0u, w);
        double dx1 = U01_LOW(w[0]), dx2 = U01_LOW(w[1]);
        orc_metric mp;
        orc_metric_at(p, i + dx1, j + dx2, 1, &mp);
        for (int s = 0; s < 2; ++s) {
          int64_t q = q0 + s;
          double uh[3], u[3];
          mj_sample(seed, (uint32_t)(2 * k + s), sub, T, uh);
          orc_hat_to_cov(&mp, uh, u);
          P->i1[q] = i; P->i2[q] = j; P->dx1[q] = dx1; P->dx2[q] = dx2;
          P->i1p[q] = i; P->i2p[q] = j; P->dx1p[q] = dx1; P->dx2p[q] = dx2;
          P->u1[q] = u[0]; P->u2[q] = u[1]; P->u3[q] = u[2];
          P->w[q] = w_inj; P->phi[q] = 0.0;
          P->tag[q] = (uint8_t)(s == 0 ? 1 : 2);
        }
      }
    }
  }
  free(wsum);
  return k;
}

/* magnetisation sigma of every cell (the quantity the injection tests;
 * +infinity in a magnetised empty cell, 0 where B = 0), written to an
 * n_r x n_th array */
void orc_magnetisation(const orc_params* p, const double* F, const orc_particles* P, double* sigma)
{
  double* wsum = cell_weights(p, P);
  for (int i = 0; i < p->n_r; ++i)
    for (int j = 0; j < p->n_th; ++j) {
      double bb, n;
      cell_magnetisation(p, F, wsum, i, j, &bb, &n);
      sigma[(int64_t)i * p->n_th + j] = bb <= 0.0 ? 0.0 : (n > 0.0 ? bb / (4.0 * M_PI * n) : INFINITY);
    }
  free(wsum);
}

/* ------------------------------------------------------ diagnostics */

/* Conserved energy and angular momentum per particle (Sec. 2.3):
 *   E = -u_0 - (q/m) A_0 = alpha gamma - beta^1 u_1 - (q/m) A_0,
 *   L = u_3 + (q/m) A_3,
 * evaluated at the time-centred position (midpoint of the previous and current
 * positions, Sec. 4.1) with theta clamped; A from the Wald potential of
 * amplitude B0 (zero for B0 = 0).  Dead slots give NaN. */
void orc_energy_momentum(const orc_params* p, const orc_particles* P, double B0v, double* E,
                         double* L)
{
  for (int64_t k = 0; k < P->n; ++k) {
    if (P->tag[k] == 0) { E[k] = NAN; L[k] = NAN; continue; }
    double x1 = 0.5 * ((P->i1p[k] + P->dx1p[k]) + (P->i1[k] + P->dx1[k]));
    double x2 = 0.5 * ((P->i2p[k] + P->dx2p[k]) + (P->i2[k] + P->dx2[k]));
    orc_metric m;
    orc_metric_at(p, x1, x2, 1, &m);
    double u[3] = {P->u1[k], P->u2[k], P->u3[k]};
    double qm = tag_qm(P->tag[k]);
    orc_wald w;
    wald_at(p, m.r, m.th, B0v, &w);
    E[k] = m.alpha * gamma_m(&m, u, tag_mass2(P->tag[k])) - m.beta1 * u[0] - qm * w.A0;
    L[k] = u[2] + qm * w.A3;
  }
}

/* Gauss-law residual at nodes (Sec. 3.2): res(i, j) = Delta_i(sqrt(h) D^1)
 * + Delta_j(sqrt(h) D^2) - 4 pi (sqrt(h) rho), with the conformal charge of the
 * current positions (two-sided on the axis rows, like the deposit) filtered
 * like the currents (n_f passes).  On the axis nodes the polar-cap form of
 * Sec. 3.3.2: A_{i+1/2} D^1(i+1/2, 0) - A_{i-1/2} D^1(i-1/2, 0)
 * + sqrt(h) D^2(i, 1/2) - 2 pi (two-sided charge), and its mirror image at
 * theta = pi with the opposite orientation of the D^2 flux (R29).
 * Written to `res` (a plane; zero outside i in [n_f + 2, i_hi), j in [0, n_th]):
 * the horizon layer overwrites the columns i <= n_f, and the outer columns
 * from i_hi = n_r - max(n_absorb, n_f) on are the absorbing layer or take
 * filtered charge from particles that leave the grid (their charge vanishes
 * on removal without a current).  Returns the largest |res| and, in *scale,
 * the largest |term|. */
double orc_gauss_residual(const orc_params* p, const double* F, const orc_particles* P, double* res,
                          double* tmp, double* scale)
{
  const int64_t pl = g_plane(p);
  const double *D1 = F + P_D * pl, *D2 = F + (P_D + 1) * pl;
  orc_charge(p, P, tmp);
  filter_scalar(p, tmp, res);
  double* rho = (double*)malloc(sizeof(double) * pl);
  memcpy(rho, tmp, sizeof(double) * pl);
  memset(res, 0, sizeof(double) * pl);
  double mx = 0.0, sc = 0.0;
  const int nth = p->n_th;
  const int i_hi = p->n_r - (p->n_absorb > p->n_filter ? p->n_absorb : p->n_filter);
  for (int i = p->n_filter + 2; i < i_hi; ++i) {
    for (int j = 1; j < nth; ++j) {
      gpt a, b, c, d;
      grid_metric(p, i, j, 1, 0, &a);
      grid_metric(p, i - 1, j, 1, 0, &b);
      grid_metric(p, i, j, 0, 1, &c);
      grid_metric(p, i, j - 1, 0, 1, &d);
      double t1 = a.sqrt_h * D1[IX(p, i, j)], t2 = b.sqrt_h * D1[IX(p, i - 1, j)];
      double t3 = c.sqrt_h * D2[IX(p, i, j)], t4 = d.sqrt_h * D2[IX(p, i, j - 1)];
      double t5 = 4.0 * M_PI * rho[IX(p, i, j)];
      double r = (t1 - t2) + (t3 - t4) - t5;
      res[IX(p, i, j)] = r;
      if (fabs(r) > mx) mx = fabs(r);
      double tm = fmax(fmax(fabs(t1), fabs(t2)), fmax(fmax(fabs(t3), fabs(t4)), fabs(t5)));
      if (tm > sc) sc = tm;
    }
    const double Ahi = polar_area(p, i), Alo = polar_area(p, i - 1);
    for (int side = 0; side < 2; ++side) {
      const int j = side ? nth : 0;
      gpt c;
      grid_metric(p, i, side ? nth - 1 : 0, 0, 1, &c);
      double t1 = Ahi * D1[IX(p, i, j)], t2 = Alo * D1[IX(p, i - 1, j)];
      double t3 = c.sqrt_h * D2[IX(p, i, side ? nth - 1 : 0)];
      double t5 = 2.0 * M_PI * rho[IX(p, i, j)];
      double r = (t1 - t2) + (side ? -t3 : t3) - t5;
      res[IX(p, i, j)] = r;
      if (fabs(r) > mx) mx = fabs(r);
      double tm = fmax(fmax(fabs(t1), fabs(t2)), fmax(fabs(t3), fabs(t5)));
      if (tm > sc) sc = tm;
    }
  }
  free(rho);
  *scale = sc;
  return mx;
}

/* dt by the Courant rule of reading R20: the largest coordinate speed of light
 * over the cell centres, |v1| <= alpha sqrt(h^11) + |beta^1|, |v2| <= alpha
 * sqrt(h^22), dt = cfl / max sqrt(v1^2 + v2^2).  Uses theta clamping. */
double orc_courant_dt(const orc_params* p, double cfl)
{
  double vmax = 0.0;
  for (int i = 0; i < p->n_r; ++i)
    for (int j = 0; j < p->n_th; ++j) {
      orc_metric m;
      orc_metric_at(p, i + 0.5, j + 0.5, 1, &m);
      double v1 = m.alpha * sqrt(m.hu11) + fabs(m.beta1);
      double v2 = m.alpha * sqrt(m.hu22);
      double v = sqrt(v1 * v1 + v2 * v2);
      if (v > vmax) vmax = v;
    }
  return cfl / vmax;
}

/* ------------------------------------------------- parts, for the pins */

/* The parts below are called on their own by the tests that pin them. */

/* gather of Sec. 3.1 step 2 at a position: D^n from plane P_D, B^n from P_B0 */
void orc_gather(const orc_params* p, const double* F, int i1, double dx1, int i2, double dx2,
                double D[3], double B[3])
{
  const int64_t pl = g_plane(p);
  gather(p, F + P_D * pl, F + P_B0 * pl, i1, dx1, i2, dx2, D, B);
}

/* axis reflection of a triple (kind 0 D-like, 1 B-like, 2 current) */
void orc_axis_bc(const orc_params* p, double* X, int kind) { axis_bc(p, X, kind); }

/* boundaries of an updated triple against its absorbing-layer target */
void orc_field_bc(const orc_params* p, double* X, const double* Xinit, int kind)
{
  field_bc(p, X, Xinit, kind);
}

/* the n_f filter passes on the current planes P_J */
void orc_filter_currents(const orc_params* p, double* F) { filter_currents(p, F); }

/* absorbing-layer ramp lambda at x1 = x */
double orc_match_lambda(const orc_params* p, double x) { return match_lambda(p, x); }

