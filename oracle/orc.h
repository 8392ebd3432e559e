/*
 * orc.h -- FP64 CPU oracle for the MRT lattice Boltzmann model of double-diffusive
 * convection in fluid-saturated porous media (Liu & He, arXiv 1708.07525).
 *
 * TEST INFRASTRUCTURE ONLY.  This oracle exists to check the GPU library; only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Every quantity is double precision.  The collision is done with the explicit
 * transformation matrices M (Eq. 13) and N (Eq. 23) and their inverses, as dense
 * matrix-vector products, exactly in the order of Eqs. (10)-(11) and (21)-(22).
 *
 * Layout of every host field array: ny rows of nx values, x fastest (index y*nx + x).
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* kinds of a side of the rectangular domain.  0-2: wall half a spacing outside the first
 * node (bounce-back rules); 4-7: wall through the first node, whose populations are set by
 * the non-equilibrium extrapolation of Eqs. (33)-(35), with T and C fixed (hot/cold), from
 * the zero-flux extrapolation of Eqs. (36)-(37), or from the convective (Robin) condition of
 * Eq. (39) through Eqs. (36)-(37). */
enum {
  ORC_SIDE_HOT = 0, ORC_SIDE_COLD = 1, ORC_SIDE_ADIABATIC = 2, ORC_SIDE_PERIODIC = 3,
  ORC_SIDE_NEE_HOT = 4, ORC_SIDE_NEE_COLD = 5, ORC_SIDE_NEE_ADIABATIC = 6, ORC_SIDE_NEE_ROBIN = 7
};
/* side order */
enum { ORC_LEFT = 0, ORC_RIGHT = 1, ORC_BOTTOM = 2, ORC_TOP = 3 };
/* deliberate mistakes a test can plant in the oracle to show that a pin catches them */
enum {
  ORC_MUT_NONE = 0,
  ORC_MUT_NO_SOURCE = 1,      /* drop the D2Q5 source term of Eq. (27)                  */
  ORC_MUT_NO_HALF_FORCE = 2,  /* u from Eq. (17) without the half-step force            */
  ORC_MUT_RHO_IN_MEQ = 3,     /* rho instead of rho0 in the velocity terms of Eq. (14)  */
  ORC_MUT_BUOY_SIGN = 4,      /* flip the sign of the buoyancy of Eq. (6)               */
  ORC_MUT_MODEL_A_DIFF = 5,   /* present equilibria but Model-A diffusivity mapping     */
  ORC_MUT_NO_FORCH = 6,       /* drop the Forchheimer term of Eq. (5)                   */
  ORC_MUT_WALL_CONST = 7,     /* anti-bounce-back constant w_i*T_w instead of 2*w_i*T_w */
  ORC_MUT_ERGUN_EXP = 8,      /* phi^2 instead of phi^3 under the root of Eq. (7)       */
  ORC_MUT_WALL_VEL = 9,       /* moving-wall term of the bounce-back halved             */
  ORC_MUT_MODEL_A_MAP = 10,   /* Model-A equilibria with the present diffusivity mapping */
  ORC_MUT_NEE_WALL_VEL = 11   /* node walls: equilibrium of Eq. (33) at rest, not the wall's velocity */
};

typedef struct orc_params {
  int32_t nx, ny;
  int32_t model;      /* 0: present model, Eqs. (24)-(25), (29); 1: Model-A, Eqs. (30)-(32) */
  int32_t mutation;   /* ORC_MUT_*, 0 in every real use */
  int32_t side[4];    /* ORC_SIDE_* for left, right, bottom, top */
  double Ra, Pr, Le, Da, N;   /* dimensionless groups of section 2 */
  double J, sigma, phi;       /* viscosity ratio, heat-capacity ratio, uniform porosity */
  double Ma, varpi, rho0;     /* Mach number (section 4.1), model parameter of Eq. (24) (<=0: auto), rho0 */
  double s_rho, s_e, s_eps, s_j, s_q;           /* D2Q9 free rates (section 4) */
  double zeta0, zeta_e, zeta_eps, eta0, eta_e, eta_eps;  /* D2Q5 free rates */
  double Th, Tl, Ch, Cl;      /* hot/cold wall temperature and concentration */
  double Fphi;                /* < 0: Ergun, Eq. (7); >= 0: this value everywhere */
  double g_ext[2];            /* extra constant body acceleration added to G */
  double wall_u[4];           /* tangential velocity of each side (moving lid) */
  int32_t direct;             /* 0: map Ra, Pr, Le, Da, N, Ma to lattice units as in section 4.1;
                                 1: take the lattice values below as given;
                                 2: lid-driven mixed convection of section 4.3: map Re, Gr, U0
                                    (with Pr, Le, Da, N) */
  double nu, alpha_e, D_e, K, gbT, gbC;  /* lattice viscosity, diffusivities, mean permeability,
                                            g*beta_T and g*beta_C, used when direct == 1 */
  double Bi_T, Bi_C;          /* Biot numbers of a convective side (Eq. 39); ambient Tl, Cl */
  double Re, Gr, U0;          /* Reynolds and Grashof numbers and the lid speed (direct == 2) */
  int32_t nee_link;           /* walls through the nodes, reading of Eq. (33): 0: every population
                                 of the boundary node from the neighbour along the inward normal;
                                 1: only the populations streaming in from outside, each from
                                 the neighbour along its own link, x_f = x_b + e_i */
} orc_params;

typedef struct orc orc;

/* derived lattice values, reported for tests */
typedef struct orc_derived {
  double L, U, nu, nu_e, alpha_e, D_e, s_v, zeta_a, eta_D, varpi, csT2;
  double gbT, gbC, T0, C0, dT, dC, K_mean, phi_min;
} orc_derived;

typedef struct orc_obs {
  int64_t step;
  double Nu[4], Sh[4];        /* per side; 0 where the side is not held at a fixed T/C */
  double mass, heat, solute;  /* sum rho, sum sigma*T, sum phi*C */
  double max_ux, max_uy;
  double r_u, r_T, r_C;       /* residuals against the last snapshot */
  int32_t nonfinite;
} orc_obs;

orc *orc_create(const orc_params *p);
/* phi may be NULL (uniform p->phi); T, C may be NULL (T0, C0); ux, uy may be NULL (0). */
int orc_set_fields(orc *o, const double *phi, const double *T, const double *C,
                   const double *ux, const double *uy);
int orc_step(orc *o, int64_t nsteps);
/* macroscopic fields at the current time level: rho, ux, uy, T, C (each nx*ny, may be NULL) */
int orc_macro(orc *o, double *rho, double *ux, double *uy, double *T, double *C);
int orc_observables(orc *o, orc_obs *out);
int orc_derived_values(const orc *o, orc_derived *out);
/* raw pre-collision populations: f (9*nx*ny), g (5*nx*ny), h (5*nx*ny); set or get */
int orc_get_populations(const orc *o, double *f, double *g, double *h);
int orc_set_populations(orc *o, const double *f, const double *g, const double *h);
void orc_destroy(orc *o);

/* building blocks exposed for the matrix-identity pins */
void orc_matrices(double *M, double *Minv, double *N, double *Ninv);
void orc_meq(double rho, double ux, double uy, double phi, double rho0, double *meq9);
void orc_feq(double rho, double ux, double uy, double phi, double rho0, double *feq9);
void orc_force_moments(double ux, double uy, double Fx, double Fy, double phi, double rho0, double *S9);
void orc_geq(double T, double ux, double uy, double cap, double varpi, int model, double *geq5);
void orc_ngeq(double T, double ux, double uy, double cap, double varpi, int model, double *neq5);
void orc_source5(double ax, double ay, double varpi, double *S5tilde);
/* porous coefficients at node k (valid after orc_set_fields): out = {K, F_phi, l0, l1} with
   l0 = (1 + phi nu/(2K))/2 and l1 = phi F_phi/(2 sqrt K) of Eq. (19) */
int orc_node_coeffs(const orc *o, long k, double *out4);
/* one velocity solve, Eqs. (18)-(19): v in, u out */
void orc_velocity(double vx, double vy, double l0, double l1, double *ux, double *uy);
int orc_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
