/* Driver for a build of the FP64 oracle (oracle/orc.c) under the address and undefined-behaviour
 * sanitizers: small lattices of every wall family, a porosity field, periodic sides, the
 * lid-driven mapping, populations set and read back, observables and derived values.  Any
 * out-of-bounds access, leak or undefined operation makes the sanitizer runtime fail the run;
 * the exit status is also non-zero when a call reports an error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "orc.h"

static orc_params base(int nx, int ny) {
  orc_params p;
  memset(&p, 0, sizeof p);
  p.nx = nx;
  p.ny = ny;
  p.side[0] = ORC_SIDE_HOT;
  p.side[1] = ORC_SIDE_COLD;
  p.side[2] = ORC_SIDE_ADIABATIC;
  p.side[3] = ORC_SIDE_ADIABATIC;
  p.Ra = 1e4; p.Pr = 1.0; p.Le = 2.0; p.Da = 1e-2; p.N = 1.0;
  p.J = 1.0; p.sigma = 1.3; p.phi = 0.6; p.Ma = 0.1; p.rho0 = 1.0;
  p.s_rho = 1.0; p.s_e = 1.1; p.s_eps = 1.1; p.s_j = 1.0; p.s_q = 1.2;
  p.zeta0 = p.eta0 = 1.0; p.zeta_e = p.zeta_eps = p.eta_e = p.eta_eps = 1.5;
  p.Th = 1.0; p.Tl = 0.0; p.Ch = 1.0; p.Cl = 0.0;
  p.Fphi = -1.0;
  return p;
}

static int run(const orc_params *p, int with_phi, int steps) {
  const int nx = p->nx, ny = p->ny;
  const long n = (long)nx * ny;
  double *phi = malloc(n * sizeof(double)), *T = malloc(n * sizeof(double)), *C = malloc(n * sizeof(double));
  double *f = malloc(9 * n * sizeof(double)), *g = malloc(5 * n * sizeof(double)), *h = malloc(5 * n * sizeof(double));
  double *F = malloc(5 * n * sizeof(double));
  int bad = 0;
  for (long k = 0; k < n; ++k) {
    phi[k] = 0.45 + 0.4 * (double)((k * 7919) % 101) / 101.0;
    T[k] = 0.5 + 1e-3 * sin((double)k);
    C[k] = 0.5 - 1e-3 * cos((double)k);
  }
  orc *o = orc_create(p);
  if (!o) { bad = 1; goto out; }
  if (orc_set_fields(o, with_phi ? phi : NULL, T, C, NULL, NULL)) bad = 1;
  if (!bad && orc_step(o, steps)) bad = 1;
  orc_obs ob;
  orc_derived d;
  double c4[4];
  if (!bad && orc_observables(o, &ob)) bad = 1;
  if (!bad && orc_derived_values(o, &d)) bad = 1;
  if (!bad && orc_node_coeffs(o, n - 1, c4)) bad = 1;
  if (!bad && orc_get_populations(o, f, g, h)) bad = 1;
  if (!bad && orc_set_populations(o, f, g, h)) bad = 1;
  if (!bad && orc_step(o, 2)) bad = 1;
  if (!bad && orc_macro(o, F, F + n, F + 2 * n, F + 3 * n, F + 4 * n)) bad = 1;
  if (!bad && (ob.nonfinite || !isfinite(F[0]))) bad = 1;
  orc_destroy(o);
out:
  free(phi); free(T); free(C); free(f); free(g); free(h); free(F);
  return bad;
}

int main(void) {
  int bad = 0;
  orc_params p = base(7, 6);
  bad |= run(&p, 0, 20);                        /* half-way walls, uniform porosity */
  bad |= run(&p, 1, 20);                        /* porosity field */
  p.model = 1;
  bad |= run(&p, 0, 10);                        /* Model-A */
  p = base(3, 3);
  bad |= run(&p, 0, 10);                        /* the smallest lattice */
  p = base(9, 8);
  p.side[0] = ORC_SIDE_NEE_HOT; p.side[1] = ORC_SIDE_NEE_ROBIN;
  p.side[2] = ORC_SIDE_NEE_ADIABATIC; p.side[3] = ORC_SIDE_NEE_COLD;
  p.Bi_T = 1.0; p.Bi_C = 5.0;
  bad |= run(&p, 1, 20);                        /* walls through the nodes, convective side */
  p = base(5, 5);
  p.side[0] = p.side[1] = ORC_SIDE_NEE_ADIABATIC; p.side[2] = p.side[3] = ORC_SIDE_PERIODIC;
  bad |= run(&p, 0, 10);                        /* node walls, periodic in y */
  p = base(6, 4);
  p.side[0] = p.side[1] = p.side[2] = p.side[3] = ORC_SIDE_PERIODIC;
  p.g_ext[0] = 1e-5;
  bad |= run(&p, 1, 10);                        /* fully periodic */
  p = base(8, 8);
  p.side[0] = p.side[1] = ORC_SIDE_ADIABATIC; p.side[2] = ORC_SIDE_COLD; p.side[3] = ORC_SIDE_HOT;
  p.direct = 2; p.Re = 100.0; p.Gr = 100.0; p.U0 = 0.1; p.wall_u[3] = 0.1;
  bad |= run(&p, 0, 20);                        /* lid-driven mapping, moving wall */
  /* rejected inputs must fail cleanly */
  p = base(2, 8);
  if (orc_create(&p)) bad = 1;
  p = base(8, 8);
  p.side[0] = ORC_SIDE_NEE_HOT;
  if (orc_create(&p)) bad = 1;
  printf(bad ? "oracle sanitize run: FAILED\n" : "oracle sanitize run: ok\n");
  return bad;
}
