/*
 * orc.c -- FP64 CPU oracle of the triple-distribution MRT lattice Boltzmann model for
 * double-diffusive convection in porous media (Liu & He, arXiv 1708.07525).
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU
 * baseline are the only users.  It is deliberately plain and slow: every node applies
 * the explicit 9x9 matrix M of Eq. (13), the diagonal relaxation matrix Lambda and
 * M^-1, and the explicit 5x5 matrix N of Eq. (23), Theta/Q and N^-1, as dense
 * matrix-vector products, in the order the paper states them.  No blocking, fusion or
 * algebraic shortcut.  Compile without fast-math and without FP contraction.
 *
 * One time step n -> n+1 (state = pre-collision populations P(n) and the products
 * T*u, C*u of step n-1):
 *   1. macroscopic fields from P(n): rho (Eq. 16), T and C (Eq. 26), the buoyancy G
 *      (Eq. 6), the explicit velocity (Eqs. 18-19) and the total force F (Eq. 5);
 *   2. D2Q9 collision in moment space, Eq. (10) with m^eq of Eq. (14) (alpha1 = 1,
 *      alpha2 = -3) and S of Eq. (15); f* = M^-1 m*;
 *   3. D2Q5 collisions of g and h, Eqs. (21)-(22), with the equilibrium moments of
 *      Eqs. (24)-(25) (or (30)-(31) for Model-A) and the source term of Eq. (27), whose
 *      time derivative is the backward difference over one step stated in section 3.2;
 *   4. save T*u and C*u of step n;
 *   5. streaming, Eq. (11), as a pull from the upstream node, with wall rules:
 *      half-way bounce-back for f (plus the moving-wall momentum term), anti-bounce-back
 *      for a side held at a fixed T/C and bounce-back for a zero-flux side, for g and h.
 *      The anti-bounce-back constant is g^eq_i + g^eq_opp(i) evaluated with the wall
 *      values, from Eq. (28).
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- lattices (Eq. 8) ---------------------------------------------------------- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* ---- transformation matrices ---------------------------------------------------- */
/* Eq. (13): rows are the moments (rho, e, eps, jx, qx, jy, qy, pxx, pxy) */
static const double M9[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};
/* Eq. (23) */
static const double N5[5][5] = {
    {1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0},
    {0, 0, 1, 0, -1},
    {-4, 1, 1, 1, 1},
    {0, 1, -1, 1, -1}};

/* The rows of M and N are mutually orthogonal (the paper states it for N; for M it is
 * the Lallemand-Luo basis), so the inverse is the transpose with each column divided by
 * the squared norm of the corresponding row. */
static double M9inv[9][9], N5inv[5][5];
static int inverses_ready = 0;

static void build_inverses(void) {
  if (inverses_ready) return;
  for (int r = 0; r < 9; ++r) {
    double nrm = 0;
    for (int c = 0; c < 9; ++c) nrm += M9[r][c] * M9[r][c];
    for (int c = 0; c < 9; ++c) M9inv[c][r] = M9[r][c] / nrm;
  }
  for (int r = 0; r < 5; ++r) {
    double nrm = 0;
    for (int c = 0; c < 5; ++c) nrm += N5[r][c] * N5[r][c];
    for (int c = 0; c < 5; ++c) N5inv[c][r] = N5[r][c] / nrm;
  }
  inverses_ready = 1;
}

static void matvec9(const double A[9][9], const double *x, double *y) {
  for (int r = 0; r < 9; ++r) {
    double s = 0;
    for (int c = 0; c < 9; ++c) s += A[r][c] * x[c];
    y[r] = s;
  }
}
static void matvec5(const double A[5][5], const double *x, double *y) {
  for (int r = 0; r < 5; ++r) {
    double s = 0;
    for (int c = 0; c < 5; ++c) s += A[r][c] * x[c];
    y[r] = s;
  }
}

/* ---- the paper's formulas, one function each ----------------------------------- */

/* Eq. (14) with alpha1 = 1, alpha2 = -3 (the values stated with Eq. 20). */
static void meq9(double rho, double ux, double uy, double phi, double rho0, int mut, double *m) {
  double rv = (mut == ORC_MUT_RHO_IN_MEQ) ? rho : rho0;
  double u2 = ux * ux + uy * uy;
  m[0] = rho;
  m[1] = -2.0 * rho + 3.0 * rv * u2 / phi;
  m[2] = 1.0 * rho - 3.0 * rv * u2 / phi;
  m[3] = rv * ux;
  m[4] = -rv * ux;
  m[5] = rv * uy;
  m[6] = -rv * uy;
  m[7] = rv * (ux * ux - uy * uy) / phi;
  m[8] = rv * ux * uy / phi;
}

/* Eq. (15). */
static void smom9(double ux, double uy, double Fx, double Fy, double phi, double rho0, double *S) {
  double uF = ux * Fx + uy * Fy;
  S[0] = 0.0;
  S[1] = 6.0 * rho0 * uF / phi;
  S[2] = -6.0 * rho0 * uF / phi;
  S[3] = rho0 * Fx;
  S[4] = -rho0 * Fx;
  S[5] = rho0 * Fy;
  S[6] = -rho0 * Fy;
  S[7] = 2.0 * rho0 * (ux * Fx - uy * Fy) / phi;
  S[8] = rho0 * (ux * Fy + uy * Fx) / phi;
}

/* Eq. (20), c_s^2 = 1/3. */
static void feq9(double rho, double ux, double uy, double phi, double rho0, double *f) {
  const double cs2 = 1.0 / 3.0;
  double u2 = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double eu = EX[i] * ux + EY[i] * uy;
    f[i] = W9[i] * (rho + rho0 * (eu / cs2 + eu * eu / (2.0 * phi * cs2 * cs2) - u2 / (2.0 * phi * cs2)));
  }
}

/* D2Q5 weights of Eq. (27): w0 = 1 - varpi, w1..4 = varpi/4. */
static double w5(int i, double varpi) { return i == 0 ? 1.0 - varpi : 0.25 * varpi; }

/* Eq. (28) (present model) or the Model-A equilibria stated after Eq. (31).
 * cap is sigma for g and phi for h. */
static void geq5(double T, double ux, double uy, double cap, double varpi, int model, double *g) {
  double csT2 = 0.5 * varpi;
  if (model == 0) {
    g[0] = cap * T - (1.0 - w5(0, varpi)) * T;
    for (int i = 1; i < 5; ++i) {
      double eu = EX[i] * ux + EY[i] * uy;
      g[i] = w5(i, varpi) * T * (1.0 + eu / csT2);
    }
  } else {
    for (int i = 0; i < 5; ++i) {
      double eu = EX[i] * ux + EY[i] * uy;
      g[i] = w5(i, varpi) * T * (cap + eu / csT2);
    }
  }
}

/* Eqs. (24)-(25) (present model) or (30)-(31) (Model-A). */
static void ngeq5(double T, double ux, double uy, double cap, double varpi, int model, double *n) {
  n[0] = cap * T;
  n[1] = ux * T;
  n[2] = uy * T;
  n[3] = (model == 0) ? (-4.0 * cap * T + 5.0 * varpi * T) : (-4.0 + 5.0 * varpi) * cap * T;
  n[4] = 0.0;
}

/* Eq. (27) in velocity space: w_i e_i . a / c_sT^2, with a = d(T u)/dt. */
static void src5(double ax, double ay, double varpi, double *s) {
  double csT2 = 0.5 * varpi;
  for (int i = 0; i < 5; ++i) s[i] = w5(i, varpi) * (EX[i] * ax + EY[i] * ay) / csT2;
}

/* Eq. (18). */
static void velocity(double vx, double vy, double l0, double l1, double *ux, double *uy) {
  double vn = sqrt(vx * vx + vy * vy);
  double den = l0 + sqrt(l0 * l0 + l1 * vn);
  *ux = vx / den;
  *uy = vy / den;
}

/* ---- state --------------------------------------------------------------------- */
struct orc {
  orc_params p;
  int nee;            /* walls through the boundary nodes (kinds 4-7) */
  int nx, ny;
  long nn;
  int ready;
  int64_t step;
  /* derived */
  double L, U, nu, nu_e, alpha_e, D_e, s_v, zeta_a, eta_D, varpi, csT2;
  double gbT, gbC, T0, C0, dT, dC, K_mean, phi_min;
  double lam9[9], theta5[5];
  /* fields */
  double *phi, *K, *Fphi, *etaD;            /* per node porosity, permeability, Forchheimer, Model-A eta_D */
  double *f, *g, *h;                        /* pre-collision P(n): [i*nn + node] */
  double *fs, *gs, *hs;                     /* post-collision */
  double *Tu, *Cu;                          /* products of step n-1: [2*node + {0,1}] */
  double *snap_u, *snap_T, *snap_C;         /* residual snapshot */
  int64_t snap_step;
};

static void *xcalloc(size_t n, size_t s) {
  void *p = calloc(n ? n : 1, s);
  return p;
}

orc *orc_create(const orc_params *p) {
  build_inverses();
  if (!p || p->nx < 3 || p->ny < 3) return NULL;
  /* either every non-periodic side is a half-way wall (0-2) or every one is a wall through
     the boundary nodes (4-7) */
  int n_half = 0, n_node = 0;
  for (int s = 0; s < 4; ++s) {
    if (p->side[s] < 0 || p->side[s] > 7) return NULL;
    if (p->side[s] <= 2) n_half++;
    else if (p->side[s] >= 4) n_node++;
  }
  if (n_half && n_node) return NULL;
  /* a node wall needs two more nodes inward (f and ff) before the opposite wall */
  if (n_node && p->side[ORC_LEFT] != ORC_SIDE_PERIODIC && p->nx < 5) return NULL;
  if (n_node && p->side[ORC_BOTTOM] != ORC_SIDE_PERIODIC && p->ny < 5) return NULL;
  orc *o = (orc *)xcalloc(1, sizeof(orc));
  if (!o) return NULL;
  o->p = *p;
  o->nee = n_node > 0;
  o->nx = p->nx;
  o->ny = p->ny;
  o->nn = (long)p->nx * p->ny;
  long nn = o->nn;
  o->phi = xcalloc(nn, sizeof(double));
  o->K = xcalloc(nn, sizeof(double));
  o->Fphi = xcalloc(nn, sizeof(double));
  o->etaD = xcalloc(nn, sizeof(double));
  o->f = xcalloc(9 * nn, sizeof(double));
  o->g = xcalloc(5 * nn, sizeof(double));
  o->h = xcalloc(5 * nn, sizeof(double));
  o->fs = xcalloc(9 * nn, sizeof(double));
  o->gs = xcalloc(5 * nn, sizeof(double));
  o->hs = xcalloc(5 * nn, sizeof(double));
  o->Tu = xcalloc(2 * nn, sizeof(double));
  o->Cu = xcalloc(2 * nn, sizeof(double));
  o->snap_u = xcalloc(2 * nn, sizeof(double));
  o->snap_T = xcalloc(nn, sizeof(double));
  o->snap_C = xcalloc(nn, sizeof(double));
  if (!o->phi || !o->K || !o->Fphi || !o->etaD || !o->f || !o->g || !o->h || !o->fs || !o->gs ||
      !o->hs || !o->Tu || !o->Cu || !o->snap_u || !o->snap_T || !o->snap_C) {
    orc_destroy(o);
    return NULL;
  }
  return o;
}

void orc_destroy(orc *o) {
  if (!o) return;
  free(o->phi); free(o->K); free(o->Fphi); free(o->etaD);
  free(o->f); free(o->g); free(o->h); free(o->fs); free(o->gs); free(o->hs);
  free(o->Tu); free(o->Cu); free(o->snap_u); free(o->snap_T); free(o->snap_C);
  free(o);
}

/* Parameter mapping of sections 2 and 4.1, done once the porosity field is known. */
static int derive(orc *o) {
  const orc_params *p = &o->p;
  const double cs2 = 1.0 / 3.0;
  /* the cavity width: nx for walls half a spacing outside, nx - 1 for walls through nodes */
  o->L = o->nee ? o->nx - 1 : o->nx;
  o->dT = p->Th - p->Tl;
  o->T0 = 0.5 * (p->Th + p->Tl);
  o->dC = p->Ch - p->Cl;
  o->C0 = 0.5 * (p->Ch + p->Cl);
  if (p->direct == 2) {
    /* section 4.3, mixed convection in a lid-driven cavity: Re = U0 L/nu, so that
       1/s_v = 1/2 + J L U0/(c_s^2 Re); Gr = g beta_T dT L^3/nu^2; Pr = nu/alpha_e,
       Le = alpha_e/D_e, Da = K/L^2 and N = beta_C dC/(beta_T dT) as in section 2 */
    if (!(o->dT > 0) || !(o->dC > 0) || !(p->Re > 0) || !(p->Gr >= 0) || !(p->U0 > 0) || !(p->Pr > 0) ||
        !(p->Le > 0) || !(p->Da > 0))
      return -1;
    o->U = p->U0;
    o->nu = p->U0 * o->L / p->Re;
    o->alpha_e = o->nu / p->Pr;
    o->D_e = o->alpha_e / p->Le;
    o->K_mean = p->Da * o->L * o->L;
    o->gbT = p->Gr * o->nu * o->nu / (o->L * o->L * o->L * o->dT);
    o->gbC = p->N * o->gbT * o->dT / o->dC;
  } else if (p->direct) {
    o->nu = p->nu;
    o->alpha_e = p->alpha_e;
    o->D_e = p->D_e;
    o->K_mean = p->K;
    o->gbT = p->gbT;
    o->gbC = p->gbC;
    o->U = sqrt(fabs(o->gbT * o->dT * o->L));
  } else {
    if (!(o->dT > 0) || !(o->dC > 0) || !(p->Ra > 0) || !(p->Pr > 0) || !(p->Le > 0) || !(p->Da > 0))
      return -1;
    /* Ma = U/c_s and U = sqrt(g beta_T dT L) (section 4.1); Ra = g beta_T dT L^3/(nu alpha_e),
       Pr = nu/alpha_e, so nu = U L sqrt(Pr/Ra); Le = alpha_e/D_e; Da = K/L^2;
       N = beta_C dC/(beta_T dT). */
    o->U = p->Ma * sqrt(cs2);
    o->nu = o->U * o->L * sqrt(p->Pr / p->Ra);
    o->alpha_e = o->nu / p->Pr;
    o->D_e = o->alpha_e / p->Le;
    o->K_mean = p->Da * o->L * o->L;
    o->gbT = o->U * o->U / (o->L * o->dT);
    o->gbC = p->N * o->gbT * o->dT / o->dC;
  }
  o->nu_e = p->J * o->nu;                      /* J = nu_e/nu */
  o->s_v = 1.0 / (0.5 + o->nu_e / cs2);        /* nu_e = c_s^2 (1/s_v - 1/2) */
  double pmin = 1e300;
  for (long k = 0; k < o->nn; ++k) pmin = o->phi[k] < pmin ? o->phi[k] : pmin;
  o->phi_min = pmin;
  o->varpi = p->varpi > 0 ? p->varpi : (pmin < 0.4 ? pmin : 0.4);
  o->csT2 = 0.5 * o->varpi;
  int coupled = (p->model == 1 && p->mutation != ORC_MUT_MODEL_A_MAP) || (p->mutation == ORC_MUT_MODEL_A_DIFF);
  if (!coupled) {
    o->zeta_a = 1.0 / (0.5 + o->alpha_e / o->csT2);   /* Eq. (29) */
    o->eta_D = 1.0 / (0.5 + o->D_e / o->csT2);
  } else {
    o->zeta_a = 1.0 / (0.5 + o->alpha_e / (p->sigma * o->csT2));  /* Eq. (32) */
    o->eta_D = 1.0 / (0.5 + o->D_e / (p->phi * o->csT2));
  }
  for (long k = 0; k < o->nn; ++k)
    o->etaD[k] = coupled ? 1.0 / (0.5 + o->D_e / (o->phi[k] * o->csT2)) : o->eta_D;
  double lam[9] = {p->s_rho, p->s_e, p->s_eps, p->s_j, p->s_q, p->s_j, p->s_q, o->s_v, o->s_v};
  memcpy(o->lam9, lam, sizeof lam);
  double th[5] = {p->zeta0, o->zeta_a, o->zeta_a, p->zeta_e, p->zeta_eps};
  memcpy(o->theta5, th, sizeof th);
  return 0;
}

static void take_snapshot(orc *o);

int orc_set_fields(orc *o, const double *phi, const double *T, const double *C,
                   const double *ux, const double *uy) {
  if (!o) return -1;
  const orc_params *p = &o->p;
  long nn = o->nn;
  int uniform = (phi == NULL);
  for (long k = 0; k < nn; ++k) {
    o->phi[k] = uniform ? p->phi : phi[k];
    if (!(o->phi[k] > 0.0 && o->phi[k] <= 1.0)) return -1;
    if (!uniform && !(o->phi[k] < 1.0)) return -1;
  }
  if (derive(o)) return -1;
  /* permeability: Da L^2 for a uniform medium; for a porosity field the Kozeny-Carman
     shape of Eq. (7), K ~ phi^3/(1-phi)^2, scaled so that its mean is Da L^2 */
  if (uniform) {
    for (long k = 0; k < nn; ++k) o->K[k] = o->K_mean;
  } else {
    double s = 0;
    for (long k = 0; k < nn; ++k) {
      double q = o->phi[k];
      s += q * q * q / ((1.0 - q) * (1.0 - q));
    }
    double mean = s / nn;
    for (long k = 0; k < nn; ++k) {
      double q = o->phi[k];
      o->K[k] = o->K_mean * (q * q * q / ((1.0 - q) * (1.0 - q))) / mean;
    }
  }
  for (long k = 0; k < nn; ++k) {
    double q = o->phi[k];
    const double q3 = p->mutation == ORC_MUT_ERGUN_EXP ? q * q : q * q * q;
    o->Fphi[k] = p->Fphi >= 0 ? p->Fphi : 1.75 / sqrt(150.0 * q3);   /* Eq. (7) */
  }
  /* initial populations: Eq. (20) with rho = rho0 and Eq. (28) */
  for (long k = 0; k < nn; ++k) {
    double t = T ? T[k] : o->T0, c = C ? C[k] : o->C0;
    double vx = ux ? ux[k] : 0.0, vy = uy ? uy[k] : 0.0;
    double fe[9], ge[5], he[5];
    feq9(p->rho0, vx, vy, o->phi[k], p->rho0, fe);
    geq5(t, vx, vy, p->sigma, o->varpi, p->model, ge);
    geq5(c, vx, vy, o->phi[k], o->varpi, p->model, he);
    for (int i = 0; i < 9; ++i) o->f[i * nn + k] = fe[i];
    for (int i = 0; i < 5; ++i) o->g[i * nn + k] = ge[i];
    for (int i = 0; i < 5; ++i) o->h[i * nn + k] = he[i];
    /* products of the step before the first one: the given fields */
    o->Tu[2 * k] = t * vx;
    o->Tu[2 * k + 1] = t * vy;
    o->Cu[2 * k] = c * vx;
    o->Cu[2 * k + 1] = c * vy;
  }
  o->step = 0;
  o->ready = 1;
  take_snapshot(o);   /* the residual snapshot starts at the initial level */
  return 0;
}

/* macroscopic fields of one node from P(n) */
typedef struct {
  double rho, T, C, ux, uy, Gx, Gy, Fx, Fy;
} node_macro;

/* Darcy and Forchheimer coefficients of Eq. (5) at node k: a = phi nu/K, b = phi F_phi/sqrt(K) */
static void porous_ab(const orc *o, long k, double *a, double *b) {
  const double phi = o->phi[k];
  *a = phi * o->nu / o->K[k];
  *b = phi * o->Fphi[k] / sqrt(o->K[k]);
  if (o->p.mutation == ORC_MUT_NO_FORCH) *b = 0.0;
}

static void node_fields(const orc *o, long k, node_macro *q) {
  const orc_params *p = &o->p;
  long nn = o->nn;
  double rho = 0, jx = 0, jy = 0, sg = 0, sh = 0;
  for (int i = 0; i < 9; ++i) {
    double fi = o->f[i * nn + k];
    rho += fi;                      /* Eq. (16) */
    jx += EX[i] * fi;
    jy += EY[i] * fi;
  }
  for (int i = 0; i < 5; ++i) {
    sg += o->g[i * nn + k];
    sh += o->h[i * nn + k];
  }
  double phi = o->phi[k];
  double T = sg / p->sigma;          /* Eq. (26) */
  double C = sh / phi;
  double buoy = o->gbT * (T - o->T0) + o->gbC * (C - o->C0);   /* Eq. (6) */
  if (p->mutation == ORC_MUT_BUOY_SIGN) buoy = -buoy;
  double Gx = p->g_ext[0], Gy = p->g_ext[1] + buoy;
  double a, b;
  porous_ab(o, k, &a, &b);
  double ux, uy;
  if (p->mutation == ORC_MUT_NO_HALF_FORCE) {
    ux = jx / p->rho0;
    uy = jy / p->rho0;
  } else {
    double vx = jx / p->rho0 + 0.5 * phi * Gx;       /* Eq. (19) with delta_t = 1 */
    double vy = jy / p->rho0 + 0.5 * phi * Gy;
    double l0 = 0.5 * (1.0 + 0.5 * a);
    double l1 = 0.5 * b;
    velocity(vx, vy, l0, l1, &ux, &uy);
  }
  double un = sqrt(ux * ux + uy * uy);
  q->rho = rho;
  q->T = T;
  q->C = C;
  q->ux = ux;
  q->uy = uy;
  q->Gx = Gx;
  q->Gy = Gy;
  q->Fx = -a * ux - b * un * ux + phi * Gx;          /* Eq. (5) */
  q->Fy = -a * uy - b * un * uy + phi * Gy;
}

/* collision of one node: P(n) -> post-collision, and the products of step n */
static void collide_node(orc *o, long k) {
  const orc_params *p = &o->p;
  long nn = o->nn;
  node_macro q;
  node_fields(o, k, &q);
  double phi = o->phi[k];

  /* D2Q9, Eq. (10) */
  double f[9], m[9], meq[9], S[9], ms[9], fst[9];
  for (int i = 0; i < 9; ++i) f[i] = o->f[i * nn + k];
  matvec9(M9, f, m);
  meq9(q.rho, q.ux, q.uy, phi, p->rho0, p->mutation, meq);
  smom9(q.ux, q.uy, q.Fx, q.Fy, phi, p->rho0, S);
  for (int r = 0; r < 9; ++r) ms[r] = m[r] - o->lam9[r] * (m[r] - meq[r]) + (1.0 - 0.5 * o->lam9[r]) * S[r];
  matvec9(M9inv, ms, fst);
  for (int i = 0; i < 9; ++i) o->fs[i * nn + k] = fst[i];

  /* D2Q5 for T and C, Eqs. (21)-(22) */
  double TuX = q.T * q.ux, TuY = q.T * q.uy, CuX = q.C * q.ux, CuY = q.C * q.uy;
  for (int which = 0; which < 2; ++which) {
    const double *src = which == 0 ? o->g : o->h;
    double *dst = which == 0 ? o->gs : o->hs;
    double scal = which == 0 ? q.T : q.C;
    double cap = which == 0 ? p->sigma : phi;
    double ax = which == 0 ? TuX - o->Tu[2 * k] : CuX - o->Cu[2 * k];       /* d(Tu)/dt, backward */
    double ay = which == 0 ? TuY - o->Tu[2 * k + 1] : CuY - o->Cu[2 * k + 1];
    if (p->mutation == ORC_MUT_NO_SOURCE) ax = ay = 0.0;
    double rel[5];
    if (which == 0) {
      memcpy(rel, o->theta5, sizeof rel);
    } else {
      double r5[5] = {p->eta0, o->etaD[k], o->etaD[k], p->eta_e, p->eta_eps};
      memcpy(rel, r5, sizeof rel);
    }
    double g[5], n[5], neq[5], st[5], S5[5], ns[5], gst[5];
    for (int i = 0; i < 5; ++i) g[i] = src[i * nn + k];
    matvec5(N5, g, n);
    ngeq5(scal, q.ux, q.uy, cap, o->varpi, p->model, neq);
    src5(ax, ay, o->varpi, st);
    matvec5(N5, st, S5);                                 /* S^T = N S~ */
    for (int r = 0; r < 5; ++r) ns[r] = n[r] - rel[r] * (n[r] - neq[r]) + (1.0 - 0.5 * rel[r]) * S5[r];
    matvec5(N5inv, ns, gst);
    for (int i = 0; i < 5; ++i) dst[i * nn + k] = gst[i];
  }
  o->Tu[2 * k] = TuX;
  o->Tu[2 * k + 1] = TuY;
  o->Cu[2 * k] = CuX;
  o->Cu[2 * k + 1] = CuY;
}

/* side crossed by the D2Q5 link i whose upstream node is outside the domain */
static int side_of_link(int i) {
  switch (i) {
    case 1: return ORC_LEFT;    /* moving +x: came from x = -1 */
    case 3: return ORC_RIGHT;
    case 2: return ORC_BOTTOM;
    default: return ORC_TOP;
  }
}

static void wall_values(const orc *o, int side, double *Tw, double *Cw) {
  const orc_params *p = &o->p;
  if (p->side[side] == ORC_SIDE_HOT) {
    *Tw = p->Th;
    *Cw = p->Ch;
  } else {
    *Tw = p->Tl;
    *Cw = p->Cl;
  }
}

/* pull streaming, Eq. (11), with the wall rules, for one destination node */
static void stream_node(orc *o, int x, int y) {
  const orc_params *p = &o->p;
  const int nx = o->nx, ny = o->ny;
  const long nn = o->nn;
  const long k = (long)y * nx + x;
  const int perx = p->side[ORC_LEFT] == ORC_SIDE_PERIODIC;
  const int pery = p->side[ORC_BOTTOM] == ORC_SIDE_PERIODIC;
  const double cs2 = 1.0 / 3.0;
  for (int i = 0; i < 9; ++i) {
    int sx = x - EX[i], sy = y - EY[i];
    int outx = sx < 0 || sx >= nx, outy = sy < 0 || sy >= ny;
    if (outx && perx) { sx = (sx + nx) % nx; outx = 0; }
    if (outy && pery) { sy = (sy + ny) % ny; outy = 0; }
    if (outx || outy) {
      /* half-way bounce-back; a moving side adds 2 w_i rho0 e_i.u_w / c_s^2 */
      double uwx = 0, uwy = 0;
      if (outy) uwx = p->wall_u[sy < 0 ? ORC_BOTTOM : ORC_TOP];
      else uwy = p->wall_u[sx < 0 ? ORC_LEFT : ORC_RIGHT];
      const double mw = p->mutation == ORC_MUT_WALL_VEL ? 1.0 : 2.0;
      o->f[i * nn + k] = o->fs[OPP[i] * nn + k] + mw * W9[i] * p->rho0 * (EX[i] * uwx + EY[i] * uwy) / cs2;
    } else {
      o->f[i * nn + k] = o->fs[i * nn + (long)sy * nx + sx];
    }
  }
  for (int which = 0; which < 2; ++which) {
    double *dst = which == 0 ? o->g : o->h;
    const double *src = which == 0 ? o->gs : o->hs;
    dst[k] = src[k];
    for (int i = 1; i < 5; ++i) {
      int sx = x - EX[i], sy = y - EY[i];
      int outx = sx < 0 || sx >= nx, outy = sy < 0 || sy >= ny;
      if (outx && perx) { sx = (sx + nx) % nx; outx = 0; }
      if (outy && pery) { sy = (sy + ny) % ny; outy = 0; }
      if (!(outx || outy)) {
        dst[i * nn + k] = src[i * nn + (long)sy * nx + sx];
        continue;
      }
      int side = side_of_link(i);
      if (p->side[side] >= ORC_SIDE_NEE_HOT) {
        dst[i * nn + k] = src[OPP[i] * nn + k];   /* placeholder: replaced by the extrapolation */
      } else if (p->side[side] == ORC_SIDE_ADIABATIC) {
        dst[i * nn + k] = src[OPP[i] * nn + k];               /* zero flux: bounce-back */
      } else {
        /* fixed value: anti-bounce-back, g_i = -g*_opp + g^eq_i(w) + g^eq_opp(w) */
        double Tw, Cw;
        wall_values(o, side, &Tw, &Cw);
        double sc = which == 0 ? Tw : Cw;
        double cap = which == 0 ? p->sigma : o->phi[k];
        double uwx = (side == ORC_BOTTOM || side == ORC_TOP) ? p->wall_u[side] : 0.0;
        double uwy = (side == ORC_LEFT || side == ORC_RIGHT) ? p->wall_u[side] : 0.0;
        double ge[5];
        geq5(sc, uwx, uwy, cap, o->varpi, p->model, ge);
        double cst = ge[i] + ge[OPP[i]];
        if (p->mutation == ORC_MUT_WALL_CONST) cst = 0.5 * cst;
        dst[i * nn + k] = -src[OPP[i] * nn + k] + cst;
      }
    }
  }
}

/* Walls through the boundary nodes (section 3.3).  After streaming, every boundary node
 * takes the populations of Eqs. (33)-(35):
 *   f_i(b) = f_i^eq(rho_f, u_b) + [f_i(f) - f_i^eq(rho_f, u_f)],
 *   g_i(b) = g_i^eq(T_b, u_b) + [g_i(f) - g_i^eq(T_f, u_f)],   h likewise with C,
 * where f is the neighbouring node along the inward normal (the inward diagonal at a corner)
 * and every value on the right is the streamed (pre-collision) state of this level.  T_b is
 * the side's fixed value, or Eq. (36) with zero gradient, or Eq. (36) with the convective
 * gradient of Eq. (39) (flux out = Bi/L (T_b - T_inf)):
 *   T_b = (4 T_f - T_ff + 2 (Bi/L) T_inf) / (3 + 2 Bi/L),
 * ff being the next node inward.  A corner takes its neighbours along the inward diagonal
 * and the rule of one of its two sides, in this order: a fixed value of the left/right side,
 * of the bottom/top side, a convective left/right side, a convective bottom/top side, else
 * zero gradient (the diagonal step has unit component along each normal, so the rule of a
 * side applies unchanged when the other side carries no flux); its wall velocity is zero. */
static int is_fixed(int kind) { return kind == ORC_SIDE_NEE_HOT || kind == ORC_SIDE_NEE_COLD; }

static void boundary_scalar(const orc *o, int kind, double sf, double sff, int conc, double *sb) {
  const orc_params *p = &o->p;
  if (kind == ORC_SIDE_NEE_HOT) { *sb = conc ? p->Ch : p->Th; return; }
  if (kind == ORC_SIDE_NEE_COLD) { *sb = conc ? p->Cl : p->Tl; return; }
  double beta = 0.0, amb = 0.0;
  if (kind == ORC_SIDE_NEE_ROBIN) {
    beta = (conc ? p->Bi_C : p->Bi_T) / o->L;
    amb = conc ? p->Cl : p->Tl;
  }
  *sb = (4.0 * sf - sff + 2.0 * beta * amb) / (3.0 + 2.0 * beta);
}

static void apply_nee(orc *o) {
  const orc_params *p = &o->p;
  const int nx = o->nx, ny = o->ny;
  const long nn = o->nn;
  const int wx = p->side[ORC_LEFT] != ORC_SIDE_PERIODIC;    /* x sides are walls */
  const int wy = p->side[ORC_BOTTOM] != ORC_SIDE_PERIODIC;
  /* list of boundary nodes and their new populations, computed from the streamed state */
  long nb = 0;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x)
      if ((wx && (x == 0 || x == nx - 1)) || (wy && (y == 0 || y == ny - 1))) nb++;
  long *idx = malloc(nb * sizeof(long));
  double *val = malloc(nb * 19 * sizeof(double));
  if (!idx || !val) { free(idx); free(val); return; }
  long m = 0;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int onx = wx && (x == 0 || x == nx - 1), ony = wy && (y == 0 || y == ny - 1);
      if (!onx && !ony) continue;
      const int sx = x == 0 ? ORC_LEFT : ORC_RIGHT, sy = y == 0 ? ORC_BOTTOM : ORC_TOP;
      const int dx = onx ? (x == 0 ? 1 : -1) : 0, dy = ony ? (y == 0 ? 1 : -1) : 0;
      const long kb = (long)y * nx + x;
      const long kf = (long)(y + dy) * nx + (x + dx);
      const long kff = (long)(y + 2 * dy) * nx + (x + 2 * dx);
      node_macro qf, qff;
      node_fields(o, kf, &qf);
      node_fields(o, kff, &qff);
      double ubx = 0.0, uby = 0.0, Tb, Cb;
      if (onx && ony) {
        const int kx = p->side[sx], ky = p->side[sy];
        int kind = ORC_SIDE_NEE_ADIABATIC;
        if (is_fixed(kx)) kind = kx;
        else if (is_fixed(ky)) kind = ky;
        else if (kx == ORC_SIDE_NEE_ROBIN) kind = kx;
        else if (ky == ORC_SIDE_NEE_ROBIN) kind = ky;
        boundary_scalar(o, kind, qf.T, qff.T, 0, &Tb);
        boundary_scalar(o, kind, qf.C, qff.C, 1, &Cb);
      } else {
        const int side = onx ? sx : sy;
        const double uw = p->mutation == ORC_MUT_NEE_WALL_VEL ? 0.0 : p->wall_u[side];
        if (onx) uby = uw;
        else ubx = uw;
        boundary_scalar(o, p->side[side], qf.T, qff.T, 0, &Tb);
        boundary_scalar(o, p->side[side], qf.C, qff.C, 1, &Cb);
      }
      const double phib = o->phi[kb], phif = o->phi[kf];
      double eb[9], ef[9], gb[5], gf[5], hb[5], hf[5];
      feq9(qf.rho, ubx, uby, phib, p->rho0, eb);               /* Eq. (33) */
      feq9(qf.rho, qf.ux, qf.uy, phif, p->rho0, ef);
      geq5(Tb, ubx, uby, p->sigma, o->varpi, p->model, gb);    /* Eq. (34) */
      geq5(qf.T, qf.ux, qf.uy, p->sigma, o->varpi, p->model, gf);
      geq5(Cb, ubx, uby, phib, o->varpi, p->model, hb);        /* Eq. (35) */
      geq5(qf.C, qf.ux, qf.uy, phif, o->varpi, p->model, hf);
      idx[m] = kb;
      for (int i = 0; i < 9; ++i) val[m * 19 + i] = eb[i] + (o->f[i * nn + kf] - ef[i]);
      for (int i = 0; i < 5; ++i) val[m * 19 + 9 + i] = gb[i] + (o->g[i * nn + kf] - gf[i]);
      for (int i = 0; i < 5; ++i) val[m * 19 + 14 + i] = hb[i] + (o->h[i * nn + kf] - hf[i]);
      if (p->nee_link) {
        /* Eq. (33) read along each link: a population that streamed in from a node inside the
           domain keeps its value; one that would come from outside takes the extrapolation from
           x_f = x_b + e_i (the normal neighbour above when that node is outside too) */
        for (int i = 0; i < 9; ++i) {
          const int ux_ = x - EX[i], uy_ = y - EY[i];
          const int in_up = (ux_ >= 0 && ux_ < nx) || !wx ? ((uy_ >= 0 && uy_ < ny) || !wy) : 0;
          if (in_up) {
            val[m * 19 + i] = o->f[i * nn + kb];
            if (i < 5) {
              val[m * 19 + 9 + i] = o->g[i * nn + kb];
              val[m * 19 + 14 + i] = o->h[i * nn + kb];
            }
            continue;
          }
          const int lx = x + EX[i], ly = y + EY[i];
          if (lx < 0 || lx >= nx || ly < 0 || ly >= ny) continue;   /* keep the normal-neighbour value */
          const long kl = (long)ly * nx + lx;
          node_macro ql;
          node_fields(o, kl, &ql);
          const double phil = o->phi[kl];
          double el[9], e2[9], gl[5], g2[5], hl[5], h2[5];
          feq9(ql.rho, ubx, uby, phib, p->rho0, el);
          feq9(ql.rho, ql.ux, ql.uy, phil, p->rho0, e2);
          val[m * 19 + i] = el[i] + (o->f[i * nn + kl] - e2[i]);
          if (i < 5) {
            geq5(Tb, ubx, uby, p->sigma, o->varpi, p->model, gl);
            geq5(ql.T, ql.ux, ql.uy, p->sigma, o->varpi, p->model, g2);
            geq5(Cb, ubx, uby, phib, o->varpi, p->model, hl);
            geq5(ql.C, ql.ux, ql.uy, phil, o->varpi, p->model, h2);
            val[m * 19 + 9 + i] = gl[i] + (o->g[i * nn + kl] - g2[i]);
            val[m * 19 + 14 + i] = hl[i] + (o->h[i * nn + kl] - h2[i]);
          }
        }
      }
      m++;
    }
  for (long j = 0; j < nb; ++j) {
    for (int i = 0; i < 9; ++i) o->f[i * nn + idx[j]] = val[j * 19 + i];
    for (int i = 0; i < 5; ++i) o->g[i * nn + idx[j]] = val[j * 19 + 9 + i];
    for (int i = 0; i < 5; ++i) o->h[i * nn + idx[j]] = val[j * 19 + 14 + i];
  }
  free(idx);
  free(val);
}

int orc_step(orc *o, int64_t nsteps) {
  if (!o || !o->ready) return -1;
  const int nx = o->nx, ny = o->ny;
  /* threads only pay off on lattices large enough to amortise the fork and barrier of a
     parallel loop; tiny lattices (the pins) stay on one thread */
  const int par = (long)nx * ny >= 16384;
  for (int64_t s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static) if (par)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) collide_node(o, (long)y * nx + x);
#pragma omp parallel for schedule(static) if (par)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) stream_node(o, x, y);
    if (o->nee) apply_nee(o);
    o->step++;
  }
  return 0;
}

int orc_macro(orc *o, double *rho, double *ux, double *uy, double *T, double *C) {
  if (!o || !o->ready) return -1;
  for (long k = 0; k < o->nn; ++k) {
    node_macro q;
    node_fields(o, k, &q);
    if (rho) rho[k] = q.rho;
    if (ux) ux[k] = q.ux;
    if (uy) uy[k] = q.uy;
    if (T) T[k] = q.T;
    if (C) C[k] = q.C;
  }
  return 0;
}

/* residual snapshot of u, T, C at the current level */
static void take_snapshot(orc *o) {
  for (long k = 0; k < o->nn; ++k) {
    node_macro q;
    node_fields(o, k, &q);
    o->snap_u[2 * k] = q.ux;
    o->snap_u[2 * k + 1] = q.uy;
    o->snap_T[k] = q.T;
    o->snap_C[k] = q.C;
  }
  o->snap_step = o->step;
}

/* Mean Nusselt/Sherwood number of Eq. (38) at one side.  The wall lies half a spacing
 * outside the first node; the wall-normal gradient is the second-order one-sided
 * difference through the wall value and the first two nodes, (-8 s_w + 9 s_0 - s_1)/3
 * along the inward normal.  Sign: heat flowing from the hot to the cold side counts
 * positive; L = nx (section 4.1). */
static double wall_number(const orc *o, const double *s, int side, double sw, double ds) {
  const int nx = o->nx, ny = o->ny;
  if (ds == 0.0) return 0.0;
  int n_along = (side == ORC_LEFT || side == ORC_RIGHT) ? ny : nx;
  double sum = 0;
  for (int a = 0; a < n_along; ++a) {
    long k0, k1;
    switch (side) {
      case ORC_LEFT: k0 = (long)a * nx + 0; k1 = (long)a * nx + 1; break;
      case ORC_RIGHT: k0 = (long)a * nx + nx - 1; k1 = (long)a * nx + nx - 2; break;
      case ORC_BOTTOM: k0 = a; k1 = (long)nx + a; break;
      default: k0 = (long)(ny - 1) * nx + a; k1 = (long)(ny - 2) * nx + a; break;
    }
    double dn = (-8.0 * sw + 9.0 * s[k0] - s[k1]) / 3.0;   /* d s / d n_inward */
    double sign = o->p.side[side] == ORC_SIDE_HOT ? -1.0 : 1.0;
    sum += sign * o->L * dn / ds;
  }
  return sum / n_along;
}

/* Eq. (38) at a wall through the boundary nodes: second-order one-sided gradient
 * (-3 s_b + 4 s_1 - s_2)/2 along the inward normal, trapezoidal mean along the wall.  Heat
 * leaving through a cold or convective side counts positive, as at a hot side entering. */
static double wall_number_nodes(const orc *o, const double *s, int side, double ds) {
  const int nx = o->nx, ny = o->ny;
  const int kind = o->p.side[side];
  if (ds == 0.0 || kind == ORC_SIDE_NEE_ADIABATIC) return 0.0;
  const double sign = kind == ORC_SIDE_NEE_HOT ? -1.0 : 1.0;
  int n_along = (side == ORC_LEFT || side == ORC_RIGHT) ? ny : nx;
  double sum = 0.0;
  for (int a = 0; a < n_along; ++a) {
    long k0, k1, k2;
    switch (side) {
      case ORC_LEFT: k0 = (long)a * nx; k1 = k0 + 1; k2 = k0 + 2; break;
      case ORC_RIGHT: k0 = (long)a * nx + nx - 1; k1 = k0 - 1; k2 = k0 - 2; break;
      case ORC_BOTTOM: k0 = a; k1 = (long)nx + a; k2 = 2L * nx + a; break;
      default: k0 = (long)(ny - 1) * nx + a; k1 = k0 - nx; k2 = k0 - 2L * nx; break;
    }
    const double dn = (-3.0 * s[k0] + 4.0 * s[k1] - s[k2]) / 2.0;
    const double w = (a == 0 || a == n_along - 1) ? 0.5 : 1.0;
    sum += w * sign * o->L * dn / ds;
  }
  return sum / (n_along - 1);
}

int orc_observables(orc *o, orc_obs *out) {
  if (!o || !o->ready || !out) return -1;
  long nn = o->nn;
  double *rho = malloc(nn * sizeof(double)), *ux = malloc(nn * sizeof(double));
  double *uy = malloc(nn * sizeof(double)), *T = malloc(nn * sizeof(double));
  double *C = malloc(nn * sizeof(double));
  if (!rho || !ux || !uy || !T || !C) {
    free(rho); free(ux); free(uy); free(T); free(C);
    return -1;
  }
  orc_macro(o, rho, ux, uy, T, C);
  memset(out, 0, sizeof *out);
  out->step = o->step;
  for (int s = 0; s < 4; ++s) {
    int kind = o->p.side[s];
    if (kind == ORC_SIDE_HOT || kind == ORC_SIDE_COLD) {
      double Tw, Cw;
      wall_values(o, s, &Tw, &Cw);
      out->Nu[s] = wall_number(o, T, s, Tw, o->dT);
      out->Sh[s] = wall_number(o, C, s, Cw, o->dC);
    } else if (kind >= ORC_SIDE_NEE_HOT) {
      out->Nu[s] = wall_number_nodes(o, T, s, o->dT);
      out->Sh[s] = wall_number_nodes(o, C, s, o->dC);
    }
  }
  double du2 = 0, u2 = 0, dT2 = 0, T2 = 0, dC2 = 0, C2 = 0;
  for (long k = 0; k < nn; ++k) {
    out->mass += rho[k];
    out->heat += o->p.sigma * T[k];
    out->solute += o->phi[k] * C[k];
    if (fabs(ux[k]) > out->max_ux) out->max_ux = fabs(ux[k]);
    if (fabs(uy[k]) > out->max_uy) out->max_uy = fabs(uy[k]);
    double a = ux[k] - o->snap_u[2 * k], b = uy[k] - o->snap_u[2 * k + 1];
    du2 += a * a + b * b;
    u2 += ux[k] * ux[k] + uy[k] * uy[k];
    dT2 += (T[k] - o->snap_T[k]) * (T[k] - o->snap_T[k]);
    T2 += T[k] * T[k];
    dC2 += (C[k] - o->snap_C[k]) * (C[k] - o->snap_C[k]);
    C2 += C[k] * C[k];
    if (!isfinite(rho[k]) || !isfinite(ux[k]) || !isfinite(uy[k]) || !isfinite(T[k]) || !isfinite(C[k]))
      out->nonfinite = 1;
  }
  double dn = (double)(o->step - o->snap_step);
  if (dn > 0) {
    out->r_u = sqrt(du2) / (dn * fmax(sqrt(u2), 1e-30));
    out->r_T = sqrt(dT2) / (dn * fmax(sqrt(T2), 1e-30));
    out->r_C = sqrt(dC2) / (dn * fmax(sqrt(C2), 1e-30));
  }
  for (long k = 0; k < nn; ++k) {
    o->snap_u[2 * k] = ux[k];
    o->snap_u[2 * k + 1] = uy[k];
    o->snap_T[k] = T[k];
    o->snap_C[k] = C[k];
  }
  o->snap_step = o->step;
  free(rho); free(ux); free(uy); free(T); free(C);
  return 0;
}

int orc_derived_values(const orc *o, orc_derived *d) {
  if (!o || !d || !o->ready) return -1;
  d->L = o->L; d->U = o->U; d->nu = o->nu; d->nu_e = o->nu_e; d->alpha_e = o->alpha_e;
  d->D_e = o->D_e; d->s_v = o->s_v; d->zeta_a = o->zeta_a; d->eta_D = o->eta_D;
  d->varpi = o->varpi; d->csT2 = o->csT2; d->gbT = o->gbT; d->gbC = o->gbC;
  d->T0 = o->T0; d->C0 = o->C0; d->dT = o->dT; d->dC = o->dC; d->K_mean = o->K_mean;
  d->phi_min = o->phi_min;
  return 0;
}

int orc_node_coeffs(const orc *o, long k, double *out) {
  if (!o || !o->ready || k < 0 || k >= o->nn || !out) return -1;
  double a, b;
  porous_ab(o, k, &a, &b);
  out[0] = o->K[k];
  out[1] = o->Fphi[k];
  out[2] = 0.5 * (1.0 + 0.5 * a);   /* Eq. (19), delta_t = 1 */
  out[3] = 0.5 * b;
  return 0;
}

int orc_get_populations(const orc *o, double *f, double *g, double *h) {
  if (!o || !o->ready) return -1;
  if (f) memcpy(f, o->f, 9 * o->nn * sizeof(double));
  if (g) memcpy(g, o->g, 5 * o->nn * sizeof(double));
  if (h) memcpy(h, o->h, 5 * o->nn * sizeof(double));
  return 0;
}

int orc_set_populations(orc *o, const double *f, const double *g, const double *h) {
  if (!o || !o->ready) return -1;
  if (f) memcpy(o->f, f, 9 * o->nn * sizeof(double));
  if (g) memcpy(o->g, g, 5 * o->nn * sizeof(double));
  if (h) memcpy(o->h, h, 5 * o->nn * sizeof(double));
  return 0;
}

/* ---- building blocks for the pins ---------------------------------------------- */
void orc_matrices(double *M, double *Minv, double *N, double *Ninv) {
  build_inverses();
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) {
      if (M) M[r * 9 + c] = M9[r][c];
      if (Minv) Minv[r * 9 + c] = M9inv[r][c];
    }
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) {
      if (N) N[r * 5 + c] = N5[r][c];
      if (Ninv) Ninv[r * 5 + c] = N5inv[r][c];
    }
}
void orc_meq(double rho, double ux, double uy, double phi, double rho0, double *m) {
  meq9(rho, ux, uy, phi, rho0, ORC_MUT_NONE, m);
}
void orc_feq(double rho, double ux, double uy, double phi, double rho0, double *f) {
  feq9(rho, ux, uy, phi, rho0, f);
}
void orc_force_moments(double ux, double uy, double Fx, double Fy, double phi, double rho0, double *S) {
  smom9(ux, uy, Fx, Fy, phi, rho0, S);
}
void orc_geq(double T, double ux, double uy, double cap, double varpi, int model, double *g) {
  geq5(T, ux, uy, cap, varpi, model, g);
}
void orc_ngeq(double T, double ux, double uy, double cap, double varpi, int model, double *n) {
  ngeq5(T, ux, uy, cap, varpi, model, n);
}
void orc_source5(double ax, double ay, double varpi, double *s) { src5(ax, ay, varpi, s); }
void orc_velocity(double vx, double vy, double l0, double l1, double *ux, double *uy) {
  velocity(vx, vy, l0, l1, ux, uy);
}
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
/* threads for the following steps: n > 0 sets n, 0 restores the count at the first call */
void orc_set_threads(int n) {
#ifdef _OPENMP
  static int initial = -1;
  if (initial < 0) initial = omp_get_max_threads();
  omp_set_num_threads(n > 0 ? n : initial);
#else
  (void)n;
#endif
}
