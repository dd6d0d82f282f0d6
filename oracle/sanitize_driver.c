/*
 * Driver for a sanitizer build of the oracle (test infrastructure only).
 *
 * Includes grpic_oracle.c and calls every entry point on small grids, the
 * edge cases included: particles on both axes and both radial edges, slots
 * that leave, empty, neutral and massless slots, filter passes, the
 * absorbing layer, the general quasi-spherical map, pair injection up to the
 * capacity.  Built with -fsanitize=address,undefined it turns any access
 * outside an array (a ghost row past the end of a plane, say) or undefined
 * arithmetic into a report and a non-zero exit.
 */
#include "grpic_oracle.c"

static orc_particles alloc_particles(int64_t n)
{
  orc_particles P;
  P.n = n;
  P.i1 = calloc((size_t)n, sizeof(int32_t));
  P.i2 = calloc((size_t)n, sizeof(int32_t));
  P.i1p = calloc((size_t)n, sizeof(int32_t));
  P.i2p = calloc((size_t)n, sizeof(int32_t));
  P.dx1 = calloc((size_t)n, sizeof(double));
  P.dx2 = calloc((size_t)n, sizeof(double));
  P.dx1p = calloc((size_t)n, sizeof(double));
  P.dx2p = calloc((size_t)n, sizeof(double));
  P.u1 = calloc((size_t)n, sizeof(double));
  P.u2 = calloc((size_t)n, sizeof(double));
  P.u3 = calloc((size_t)n, sizeof(double));
  P.w = calloc((size_t)n, sizeof(double));
  P.phi = calloc((size_t)n, sizeof(double));
  P.tag = calloc((size_t)n, sizeof(uint8_t));
  return P;
}

static void free_particles(orc_particles* P)
{
  free(P->i1); free(P->i2); free(P->i1p); free(P->i2p);
  free(P->dx1); free(P->dx2); free(P->dx1p); free(P->dx2p);
  free(P->u1); free(P->u2); free(P->u3); free(P->w); free(P->phi); free(P->tag);
}

/* edge-case slots at the end of a loaded set: on both axes, at both radial
 * edges, moving out through both, neutral, massless, empty */
static void edge_slots(const orc_params* p, orc_particles* P, int64_t first)
{
  const int nr = p->n_r, nt = p->n_th;
  const int32_t ci1[8] = {0, nr - 1, nr / 2, nr / 2, 0, nr - 1, nr / 3, nr / 4};
  const int32_t ci2[8] = {nt / 2, nt / 2, 0, nt - 1, 0, nt - 1, nt / 2, nt / 3};
  const double cdx1[8] = {0.0, 0.999999, 0.5, 0.5, 1e-9, 1.0 - 1e-9, 0.3, 0.7};
  const double cdx2[8] = {0.5, 0.5, 1e-7, 1.0 - 1e-7, 0.0, 0.999999, 0.4, 0.6};
  const double cu1[8] = {-30.0, 30.0, 0.1, -0.1, -5.0, 5.0, 0.2, 0.3};
  const uint8_t ctag[8] = {1, 2, 1, 2, 2, 1, 3, 7};
  for (int k = 0; k < 8 && first + k < P->n; ++k) {
    int64_t q = first + k;
    P->i1[q] = P->i1p[q] = ci1[k];
    P->i2[q] = P->i2p[q] = ci2[k];
    P->dx1[q] = P->dx1p[q] = cdx1[k];
    P->dx2[q] = P->dx2p[q] = cdx2[k];
    P->u1[q] = cu1[k];
    P->u2[q] = 0.05 * (k - 4);
    P->u3[q] = 0.7 + 0.1 * k;
    P->w[q] = 1.0;
    P->phi[q] = 0.0;
    P->tag[q] = ctag[k];
  }
}

static int run(double a, double M, double r0, double h0, int nr, int nt, int nf, int na, int monopole)
{
  orc_params p;
  memset(&p, 0, sizeof p);
  p.a = a; p.M = M; p.r0 = r0; p.h0 = h0;
  p.r_min = M > 0.0 ? 0.9 * (M + sqrt(M * M - a * a)) : 1.0;
  p.r_max = 20.0;
  p.n_r = nr; p.n_th = nt; p.ng = 2; p.n_iter = 10;
  p.small_angle = 1e-5; p.charge_scale = 1e-3; p.n_filter = nf; p.n_absorb = na;
  p.dt = orc_courant_dt(&p, 0.5);
  const int64_t pl = orc_plane_size(&p);
  double* F = calloc((size_t)pl * ORC_NPLANE, sizeof(double));
  double* res = calloc((size_t)pl, sizeof(double));
  double* tmp = calloc((size_t)pl, sizeof(double));
  double* sig = calloc((size_t)nr * nt, sizeof(double));
  if (monopole) orc_fields_init_monopole(&p, F, 1.0);
  else orc_fields_init_wald(&p, F, 1.0);
  const int64_t n_pairs = 400, n_geo = M > 0.0 && p.r_max > 15.0 ? 20 : 0;
  const int64_t n_load = 2 * n_pairs + n_geo, n_room = 600;
  orc_particles P = alloc_particles(n_load + 8 + n_room);
  orc_particles L = P;
  L.n = n_load;
  orc_particles_init(&p, &L, n_pairs, 0, 1.0, n_geo, 7);
  edge_slots(&p, &P, n_load);
  orc_particles S = P;
  S.n = n_load + 8;                     /* loaded + edge slots, room after */
  double* E = calloc((size_t)P.n, sizeof(double));
  double* Lm = calloc((size_t)P.n, sizeof(double));
  for (int step = 0; step < 3; ++step) {
    orc_field_advance(&p, F, 0);
    orc_push(&p, F, &S);
    orc_deposit(&p, F, &S);
    orc_field_advance(&p, F, 1);
  }
  orc_charge(&p, &S, tmp);
  double scale = 0.0;
  orc_gauss_residual(&p, F, &S, res, tmp, &scale);
  orc_energy_momentum(&p, &S, 1.0, E, Lm);
  orc_magnetisation(&p, F, &S, sig);
  int64_t k = orc_inject_pairs(&p, F, &P, 1e300, 0.5, 3, 1.0, 0, nr, 5, 0, S.n);
  k += orc_inject_pairs(&p, F, &P, 1.0, 0.5, 2, 1.0, 0, nr, 5, 1, S.n + 2 * k);
  double D[3], B[3];
  orc_gather(&p, F, 0, 0.0, 0, 0.0, D, B);
  orc_gather(&p, F, nr - 1, 0.999, nt - 1, 0.999, D, B);
  orc_filter_currents(&p, F);
  for (int kind = 0; kind < 3; ++kind) orc_axis_bc(&p, F + (size_t)P_J * pl, kind);
  (void)orc_match_lambda(&p, nr - 0.5);
#ifdef PLANT_OUT_OF_BOUNDS
  /* a planted mistake for the test of the build itself: one past the set */
  F[(size_t)pl * ORC_NPLANE] += 1.0;
#endif
  free(F); free(res); free(tmp); free(sig); free(E); free(Lm);
  free_particles(&P);
  return k >= 0 ? 0 : 1;
}

int main(void)
{
  int bad = 0;
  bad |= run(0.9, 1.0, 0.0, 0.0, 24, 20, 0, 0, 0);
  bad |= run(0.9, 1.0, 0.0, 0.0, 24, 24, 3, 4, 0);
  bad |= run(0.2, 1.0, 0.4, 0.3, 20, 24, 2, 3, 1);
  bad |= run(0.95, 1.0, 0.4, -0.3, 16, 16, 4, 2, 0);
  bad |= run(0.0, 0.0, 0.0, 0.0, 16, 16, 1, 0, 0);
  return bad;
}
