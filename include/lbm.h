/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the multiple-relaxation-time lattice
 * Boltzmann model of double-diffusive convection in fluid-saturated porous media of
 * Liu & He (arXiv 1708.07525).
 *
 * One time step advances, in a single fused stream-and-collide pass over every node:
 *   - the D2Q9 flow distribution f: moment-space collision (Eq. 10) with the porous
 *     equilibrium moments (Eq. 14, alpha1 = 1, alpha2 = -3), the forcing moments (Eq. 15)
 *     of the total force of Eq. (5) (Darcy, Forchheimer, buoyancy of Eq. 6), density and
 *     the explicit velocity of Eqs. (16)-(19);
 *   - the D2Q5 temperature and concentration distributions g and h: moment-space
 *     collisions (Eqs. 21-23) with the modified equilibrium moments (Eqs. 24-25) and the
 *     source term of Eq. (27) with its time derivative taken as a one-step backward
 *     difference (section 3.2);
 *   - streaming (Eq. 11) as a pull from the upstream node, with half-way bounce-back for
 *     f, anti-bounce-back for g/h at a side held at fixed T/C and bounce-back at a zero-flux
 *     side (the constant follows from Eq. 28).
 * Parameters follow the problem statement of section 2 (Ra, Pr, Le, Da, N, J, sigma,
 * porosity) and the lattice choices of section 4 (rho0, varpi, free relaxation rates,
 * Ma = U/c_s with U = sqrt(g beta_T dT L), L = nx).
 *
 * Conventions
 *   - Host field arrays are double, ny rows of nx values, x fastest (index y*nx + x);
 *     they are borrowed for the duration of a call and copied.
 *   - Device memory belongs to the context, or to a caller arena (params.arena) that must
 *     outlive the context.
 *   - Every call returns an lbm_status; no exception crosses the ABI.  On error the
 *     context (if any) keeps a message readable with lbm_last_error().
 *   - A context is used by one host thread at a time.  Work is ordered on the context's
 *     HIP stream (params.stream, NULL = the null stream); lbm_step is asynchronous,
 *     lbm_observables and the state/field copies synchronise the stream.
 *   - Only gfx950 code is built; a context on any other device fails with LBM_EDEVICE.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* invalid argument or parameter                         */
  LBM_ENOMEM = -2,     /* device or host allocation failed, or the arena is too small */
  LBM_EDEVICE = -3,    /* HIP runtime error, or no gfx950 device                 */
  LBM_ESTATE = -4,     /* call out of order (e.g. step before set_fields)        */
  LBM_EUNSTABLE = -5   /* a non-finite value was found in the fields             */
} lbm_status;

/* Storage of the populations.  Arithmetic is FP64 for LBM_FP64 and FP32 otherwise.
 * Populations are stored as deviations from the rest state at (rho0, T0, C0): f_i - w_i rho0,
 * g_i - g_i^eq(T0, 0), h_i - h_i^eq(C0, 0).  LBM_FP16S stores them in IEEE binary16 with a
 * power-of-two pre-scale, rounded stochastically (unbiased; the random bits are a function of
 * node and step, so results are reproducible); the previous-step fields (T - T0, C - C0, u)
 * used by the source term of Eq. (27) stay FP32. */
typedef enum lbm_precision { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16S = 2 } lbm_precision;

/* Kind of a side of the rectangle.
 * 0-2: the wall lies half a spacing outside the first node.  HOT holds T = Th and C = Ch,
 *      COLD holds T = Tl and C = Cl (anti-bounce-back for g, h, constant from Eq. 28);
 *      ADIABATIC is zero flux for T and C (bounce-back).  All three are impermeable no-slip
 *      walls for f (half-way bounce-back, moving with wall_u).  L = nx.
 * 4-7: the wall passes through the first node (section 3.3): the boundary node's populations
 *      come from the non-equilibrium extrapolation of Eqs. (33)-(35) with the wall velocity
 *      wall_u and T, C fixed (NEE_HOT, NEE_COLD), extrapolated with zero gradient
 *      (NEE_ADIABATIC, Eqs. 36-37) or with the convective condition of Eq. (39)
 *      (NEE_ROBIN: flux out = Bi/L (T_b - Tl), Bi_T and Bi_C below).  L = nx - 1.
 *      Needs nx >= 5 (ny >= 5) for walls on the x (y) sides.
 * The two families cannot be mixed in one cavity.  PERIODIC must be set on both left and
 * right, or on both bottom and top. */
typedef enum lbm_side {
  LBM_SIDE_HOT = 0,
  LBM_SIDE_COLD = 1,
  LBM_SIDE_ADIABATIC = 2,
  LBM_SIDE_PERIODIC = 3,
  LBM_SIDE_NEE_HOT = 4,
  LBM_SIDE_NEE_COLD = 5,
  LBM_SIDE_NEE_ADIABATIC = 6,
  LBM_SIDE_NEE_ROBIN = 7
} lbm_side;

enum { LBM_LEFT = 0, LBM_RIGHT = 1, LBM_BOTTOM = 2, LBM_TOP = 3 };

typedef struct lbm_params {
  int32_t nx, ny;        /* lattice nodes; L = nx (or nx - 1 for walls through the nodes)  */
  int32_t precision;     /* lbm_precision                                               */
  int32_t model;         /* 0: present model (Eqs. 24-25, 29); 1: Model-A (Eqs. 30-32)    */
  int32_t side[4];       /* lbm_side of left, right, bottom, top                         */
  double Ra, Pr, Le, Da, N;   /* thermal Rayleigh, Prandtl, Lewis, Darcy, buoyancy ratio  */
  double J, sigma, phi;       /* viscosity ratio nu_e/nu, heat-capacity ratio, uniform porosity
                                 (used when lbm_set_fields gets phi == NULL)              */
  double Ma, varpi, rho0;     /* Mach number U/c_s; model parameter of Eq. (24) (<= 0:
                                 min(2/5, smallest porosity)); reference density          */
  double s_rho, s_e, s_eps, s_j, s_q;                  /* D2Q9 free rates                */
  double zeta0, zeta_e, zeta_eps, eta0, eta_e, eta_eps;  /* D2Q5 free rates              */
  double Th, Tl, Ch, Cl;      /* hot/cold T and C; dT = Th - Tl, T0 = (Th + Tl)/2, same for C */
  double Fphi;                /* < 0: Ergun, Eq. (7); >= 0: this Forchheimer coefficient  */
  double g_ext[2];            /* constant acceleration added to G of Eq. (6)              */
  double wall_u[4];           /* tangential velocity of each side (moving lid)           */
  int32_t direct;             /* how the groups map to lattice units:
                                 0: natural convection (section 4.1): Ra, Pr, Le, Da, N, Ma
                                    with U = Ma c_s = sqrt(g beta_T dT L), nu = U L sqrt(Pr/Ra);
                                 1: take nu, alpha_e, D_e, K, gbT, gbC below as lattice values;
                                 2: lid-driven mixed convection (section 4.3): Re, Gr, U0 below
                                    with Pr, Le, Da, N: nu = U0 L/Re (1/s_v = 1/2 + J L U0/(c_s^2
                                    Re)), g beta_T dT = Gr nu^2/L^3.  The moving side's speed is
                                    wall_u (U0 for the lid), set separately                  */
  double nu, alpha_e, D_e, K, gbT, gbC;
  double Bi_T, Bi_C;          /* Biot numbers of a NEE_ROBIN side (Eq. 39)                 */
  double Re, Gr, U0;          /* Reynolds and Grashof numbers, lid speed (direct == 2)     */
  void *stream;               /* hipStream_t for all work of the context (NULL: null stream) */
  void *arena;                /* optional device memory for every buffer of the context   */
  uint64_t arena_bytes;       /* size of arena; must be >= lbm_footprint_bytes()          */
} lbm_params;

/* Fills the constants of section 4: rho0 = J = sigma = 1, Ma = 0.1, varpi automatic,
 * s_rho = s_j = 1, s_e = s_eps = 1.1, s_q = 1.2, zeta0 = eta0 = 1, the other D2Q5 rates 1.5,
 * Th = Ch = 1, Tl = Cl = 0, left HOT, right COLD, bottom/top ADIABATIC, FP32, Ergun F_phi,
 * and the 64x64 porous-cavity groups nx = ny = 64, Ra = 1e4, Pr = 1, Le = 2, Da = 1e-2, N = 1,
 * phi = 0.6. */
void lbm_params_default(lbm_params *p);

/* Bytes of device memory a context with these parameters needs (for an arena). */
uint64_t lbm_footprint_bytes(const lbm_params *p);

/* Validates p, maps it to lattice units (section 4.1, Eq. 29) and allocates the device
 * buffers.  LBM_EINVAL: nx or ny < 3, a non-positive group, phi outside (0, 1], a free rate
 * outside (0, 2), a derived s_v, zeta_alpha or eta_D outside (0, 2), inconsistent periodic
 * sides, or a lattice whose 19 population planes (rows padded to 64 nodes) exceed 4 GiB in the
 * storage type (about 28M nodes in FP64, 56M in FP32, 113M in FP16: the kernels use 32-bit
 * buffer offsets).  *out is set only on LBM_OK. */
lbm_status lbm_create(const lbm_params *p, struct lbm_ctx **out);

/* Initial state from host fields (each nx*ny doubles): porosity (NULL: uniform p.phi; a
 * field must lie in (0, 1) and sets K(x) by the Kozeny-Carman form of Eq. (7) scaled to
 * mean Da L^2), T and C (NULL: T0, C0), ux and uy (NULL: 0).  The populations start at the
 * equilibria of Eqs. (20) and (28) with rho = rho0; the previous-step fields of the source
 * term start at the given T, C, u.  Resolves the automatic varpi.  Then one collision is
 * applied, so that the stored state is the post-collision populations of level 0. */
lbm_status lbm_set_fields(struct lbm_ctx *c, const double *phi, const double *T, const double *C,
                          const double *ux, const double *uy);

/* Advances nsteps >= 0 time steps (asynchronous, stream-ordered).  LBM_ESTATE before
 * lbm_set_fields, while the context is attached to a batch, or after lbm_observables has
 * reported LBM_EUNSTABLE (until lbm_set_fields or lbm_set_state gives it a new state). */
lbm_status lbm_step(struct lbm_ctx *c, int64_t nsteps);

typedef struct lbm_obs {
  int64_t step;              /* time level n of the fields                               */
  double Nu[4], Sh[4];       /* mean Nusselt / Sherwood number of Eq. (38) at each side held
                                at fixed T/C (0 elsewhere); heat flowing from hot to cold is
                                positive; second-order one-sided wall gradient           */
  double mass, heat, solute; /* sum rho, sum sigma T, sum phi C over all nodes            */
  double max_ux, max_uy;     /* largest |u_x|, |u_y|                                      */
  double r_u, r_T, r_C;      /* |X(n) - X(m)|_2 / ((n - m) max(|X(n)|_2, 1e-30)) against the
                                level m of the previous lbm_observables call (or level 0) */
  int32_t nonfinite;         /* 1 if any rho, u, T or C is NaN or infinite                */
} lbm_obs;

/* Reductions over the current level (FP64 accumulation, fixed order: the result does not
 * depend on launch shapes), optional export of the FP64 fields rho, ux, uy, T, C (5*nx*ny
 * doubles, in that order) into fields, and the residual snapshot update.  Synchronises.
 * Returns LBM_EUNSTABLE (after filling *out) when a value is not finite. */
lbm_status lbm_observables(struct lbm_ctx *c, lbm_obs *out, double *fields);

/* For callers that cannot allocate device memory (serving loops and harnesses that forbid
 * hipMalloc): lbm_observables with no allocation at all.  Same arguments, results and errors
 * as lbm_observables (the same kernels, bit for bit the same values), but the per-block partial
 * sums, the result slots and the staging of the exported fields live in a fixed device array
 * of the library (about 42 MB per device, held until the process ends) instead of the
 * context's memory and a buffer allocated per call.  Limits: at most 16384 rows (partials of
 * the reduction), and with fields != NULL at most 1048576 nodes (nx*ny); larger lattices are
 * refused with LBM_EINVAL.  Every context on a device shares that device's array and it keeps
 * the last call's contents (every value a call reads is written by the same call first): calls
 * that overlap in time on one device, from several threads or on several streams, race and must
 * be serialised by the caller.  Synchronises the context's stream. */
lbm_status lbm_observables_static(struct lbm_ctx *c, lbm_obs *out, double *fields);

/* Export of the FP64 fields rho, ux, uy, T, C of the current level (5*nx*ny doubles, in that
 * order, each ny rows of nx) without touching the residual snapshot.  Synchronises. */
lbm_status lbm_get_fields(struct lbm_ctx *c, double *fields);

/* Lattice values derived from the parameters (valid after lbm_set_fields): wall distance L,
 * velocity scale U (section 4.1) and viscosities nu, nu_e, diffusivities alpha_e, D_e, the
 * relaxation rates s_v, zeta_alpha, eta_D of Eqs. (10) and (29), varpi and c_sT^2 = varpi/2
 * (Eq. 28), g beta_T and g beta_C (Eq. 6), T0, C0, dT, dC, the mean permeability, the smallest
 * porosity and the FP16 storage pre-scale. */
typedef struct lbm_derived {
  double L, U, nu, nu_e, alpha_e, D_e, s_v, zeta_a, eta_D, varpi, csT2;
  double gbT, gbC, T0, C0, dT, dC, K_mean, phi_min, fp16_scale;
} lbm_derived;
/* Copies the context's derived values into *out (caller-owned).  LBM_EINVAL for NULL
 * arguments, LBM_ESTATE before lbm_set_fields. */
lbm_status lbm_get_derived(const struct lbm_ctx *c, lbm_derived *out);

/* The same lattice values computed on the host alone, for the uniform porosity p->phi (the
 * mapping of sections 2, 4.1 and 4.3 and Eqs. 29/32; no device is touched).  LBM_EINVAL for
 * the parameters lbm_create would refuse, or a derived rate outside (0, 2). */
lbm_status lbm_derive(const lbm_params *p, lbm_derived *out);

/* Checkpoint: the complete state (populations, previous-step fields, residual snapshot,
 * step counter).  lbm_state_bytes gives the size; lbm_get_state copies it to host memory,
 * lbm_set_state restores it into a context created with the same parameters. */
uint64_t lbm_state_bytes(const struct lbm_ctx *c);
lbm_status lbm_get_state(struct lbm_ctx *c, void *host, uint64_t bytes);
lbm_status lbm_set_state(struct lbm_ctx *c, const void *host, uint64_t bytes);

/* Launch shape of the step kernel: tile_x nodes along x (64, 128 or 256) by tile_y rows
 * (1, 2, 4 or 8) per work-group.  Results do not depend on it.  0, 0 restores the default:
 * one row of the width (256, 128 or 64) that leaves the fewest idle lanes at the right edge. */
lbm_status lbm_set_tile(struct lbm_ctx *c, int32_t tile_x, int32_t tile_y);
lbm_status lbm_get_tile(const struct lbm_ctx *c, int32_t *tile_x, int32_t *tile_y);

/* Steps per captured HIP graph replay in lbm_step: an even chunk >= 2, or 0 for one plain
 * kernel launch per step (default 64).  Results do not depend on it. */
lbm_status lbm_set_graph_chunk(struct lbm_ctx *c, int32_t chunk);

/* Cache policy of the step launch: 0 tuned per storage type on the 2048^2 cavity with one
 * step per launch (FP32: non-temporal loads, plain stores), 1 streaming (plain loads,
 * non-temporal stores), 2 resident (plain loads and stores: a step's data stays in the 256 MB
 * Infinity Cache), or -1 for the default rule: resident when a step touches at most 400 MB
 * (nx ny times 376, 188 or 112 B), else streaming, except tuned for one-step FP64 and FP16
 * launches.  Results do not depend on it.  lbm_get_cache_policy returns the policy in effect
 * (-1 for a NULL context). */
lbm_status lbm_set_cache_policy(struct lbm_ctx *c, int32_t policy);
int32_t lbm_get_cache_policy(const struct lbm_ctx *c);

/* Order in which the two- and three-step launches visit their tiles: 0 row by row of tiles,
 * k >= 1 in vertical strips k tiles wide (the last one narrower), each walked row by row, so
 * that the halo rows a tile reads were loaded shortly before by its neighbour in the strip and
 * are still in the L2 of its XCD; -1 the default rule: row by row up to 8 tiles across and
 * where a step touches at most 400 MB (the lattice stays in the Infinity Cache); otherwise for
 * three-step launches and two-step launches on 12-row tiles one strip per XCD band (tiles across
 * / 8, halved while above 8) when the tiles across are a multiple of 8, else strips of 8 tiles;
 * two-step launches on 8-row tiles row by row up to 32 tiles
 * across, strips of 8 beyond.  LBM_EINVAL outside -1..1024.  Results do not depend on it (bit for
 * bit).
 * lbm_get_strip_width returns the width in effect (-1 for a NULL context). */
lbm_status lbm_set_strip_width(struct lbm_ctx *c, int32_t tiles);
int32_t lbm_get_strip_width(const struct lbm_ctx *c);

/* Rows of the multi-step tile of the FP32 three-step and the FP16 two-step launch: 8 (64 x 8 nodes)
 * or 12 (64 x 12: fewer halo collisions per update, two work-groups per CU instead of three), or
 * 0 for the default rule (12 where a step touches more than 400 MB, i.e. the lattice streams from
 * HBM, else 8).  FP64 (32 x 8) and the node-wall launches have 8-row tiles only.  LBM_EINVAL for
 * other values (12 with FP64 storage).  Results do not depend on it (bit for bit).
 * lbm_get_tile_rows returns the rows of the multi-step launch in effect (8 for the other launches
 * and for one step per launch; 0 for a NULL context). */
lbm_status lbm_set_tile_rows(struct lbm_ctx *c, int32_t rows);
int32_t lbm_get_tile_rows(const struct lbm_ctx *c);

/* Time steps per kernel launch: 1 (step_kernel), 2 (the two-step kernel: 64 x 8 tiles, 32 x 8
 * for FP64, FP16 tiles of lbm_set_tile_rows rows, and a one-node halo staged in LDS, so the
 * global loads of the second step are saved), 3 (the three-step kernel: a two-node halo, FP32
 * tiles of lbm_set_tile_rows rows; FP32 and FP64 storage with walls half a spacing outside,
 * else 2), or 0 for the default (2 for FP16 storage, else 3).  Walls through the nodes take 1 with FP16 storage, or when the lattice is smaller than one
 * two-step tile; otherwise the two-step kernel applies the boundary rule in both steps (its last
 * tiles sit against the far walls).  Remaining steps run in shorter launches.  Results do not
 * depend on it (bit for bit).  With 3, a graph replay covers the largest multiple of 6 steps in the
 * graph chunk.  lbm_get_steps_per_launch returns the count in effect (0 for a NULL context). */
lbm_status lbm_set_steps_per_launch(struct lbm_ctx *c, int32_t n);
int32_t lbm_get_steps_per_launch(const struct lbm_ctx *c);

/* Times every supported launch shape, cache policy and steps-per-launch count on this
 * context for `steps` steps each (HIP events), the multi-step launches also with their tiles
 * row by row, in strips of 4 and 8 tiles and of one strip per XCD band, and the FP32 three-step
 * and FP16 two-step launches on
 * both their tiles,
 * keeps the fastest (read the choices with lbm_get_cache_policy, lbm_get_steps_per_launch,
 * lbm_get_strip_width, lbm_get_tile_rows),
 * restores the state it started from, and reports the tile and its time per step.
 * Synchronises. */
lbm_status lbm_autotune(struct lbm_ctx *c, int32_t steps, int32_t *tile_x, int32_t *tile_y,
                        double *ms_per_step);

/* Text of the last error on this context ("" if none); a static text for c == NULL. */
const char *lbm_last_error(const struct lbm_ctx *c);

/* Frees the context and its device memory.  NULL is a no-op.  A context still attached to a
 * batch is detached first, once the work queued on the batch's stream has finished. */
void lbm_destroy(struct lbm_ctx *c);

/* ---- batched stepping of many independent cavities --------------------------------
 * A batch advances every attached context (any size, parameters and precision).  The
 * attached contexts are split per precision and size class (width <= 64, <= 128, <= 256 or
 * wider; attach order within a class) into groups whose step touches at most 200 MB together
 * (a larger context is a group of its own); each group advances `chunk` steps before the next
 * group starts, so its data stays in the 256 MB Infinity Cache from step to step.  With an
 * even chunk that is a multiple of 4 a launch advances two steps (the two-step kernel over
 * tiles of the group's shape: 64 x 8, 32 x 16 or 32 x 8 nodes; FP64 32 x 8, 16 x 16 or 16 x 8),
 * otherwise one.  With a chunk that is a multiple of 12, FP32 and FP64 groups may instead
 * advance three steps per launch (shape index 3: the three-step kernel over the tiles of shape
 * 0).  Steps that do not fill a launch run one per launch.  A group takes the tile shape and
 * cache policy lbm_batch_autotune chose for
 * its precision and size class, or by default the first shape and the default cache-policy
 * rule of lbm_set_cache_policy for the group's bytes.  Each launch walks a device-side table of
 * (cavity, tile) work items and the launches are replayed from a captured HIP graph;
 * attaching or detaching contexts rewrites the tables between replays and re-captures only
 * when the groups' number, precisions, shapes, policies or grids change.  Per-node arithmetic
 * is the same code as lbm_step: a cavity's state after n batched steps is bitwise the state
 * after lbm_step(c, n), whatever the tile shape. */
typedef struct lbm_batch lbm_batch;

/* max_cavities: capacity of the table; chunk: steps per graph replay (even, >= 2);
 * stream: hipStream_t the batch runs on (NULL: null stream). */
lbm_status lbm_batch_create(int32_t max_cavities, int32_t chunk, void *stream, lbm_batch **out);
/* The context must be initialised (lbm_set_fields), on the batch's device and not in
 * another batch; its work moves to the batch's stream until detached.  A context with walls
 * through the boundary nodes (LBM_NEE_* sides) joins groups of its own, which advance two
 * steps per launch on the two-step tile with the last tiles against the far walls (as
 * lbm_step does); a remaining single step runs as the context's own one-step launch.  Such a
 * context is refused with LBM_EINVAL when its storage is FP16, when its lattice is smaller
 * than one two-step tile (64 x 8, FP64 32 x 8), or when the batch's chunk is not a multiple
 * of 4; it then advances with lbm_step only. */
lbm_status lbm_batch_attach(lbm_batch *b, struct lbm_ctx *c);
/* Removes the context once the work queued on the batch's stream has finished; its work
 * returns to its own stream and lbm_step applies again.  LBM_EINVAL if it is not in this batch. */
lbm_status lbm_batch_detach(lbm_batch *b, struct lbm_ctx *c);
/* Advances every attached context by nsteps (asynchronous, on the batch's stream).  LBM_EINVAL
 * for nsteps < 0, LBM_ENOMEM when the work tables cannot grow, LBM_EDEVICE on a HIP error. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);
/* Autotuner of the batched launch: for every precision and size class present, times each
 * tile shape of the two-step launch (and three steps per launch, shape 3, where the chunk and
 * the precision allow it) and each cache policy on that class's groups (`steps` steps, rounded
 * up to a multiple of 12, after a warm-up of 12), keeps the fastest, and restores
 * every attached state it started from.  shape_out and policy_out (each 12 int32, index
 * precision * 4 + size class; may be NULL) receive the choices of the classes present.
 * Synchronises; allocates a temporary device copy of the attached states. */
lbm_status lbm_batch_autotune(lbm_batch *b, int32_t steps, int32_t *shape_out, int32_t *policy_out);
/* Sets the launch choice of one precision (lbm_precision) and size class (0-3: width <= 64,
 * <= 128, <= 256, wider) without timing (e.g. from a cache of lbm_batch_autotune results):
 * shape 0-2 (two-step tiles) or 3 (three steps per launch; FP32 and FP64 only; taken as shape 0
 * with two steps per launch while the chunk is not a multiple of 12), policy 0-2 or -1 for the
 * default rule.  Takes effect at the next lbm_batch_step.  LBM_EINVAL for an index out of
 * range and for shape 3 with FP16 storage. */
lbm_status lbm_batch_set_tile(lbm_batch *b, int32_t precision, int32_t size_class, int32_t shape, int32_t policy);
/* Number of attached contexts (0 for NULL). */
int32_t lbm_batch_size(const lbm_batch *b);
/* Frees the batch once the work queued on its stream has finished; the attached contexts are
 * released to their own streams and stay valid.  NULL is a no-op. */
void lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif
