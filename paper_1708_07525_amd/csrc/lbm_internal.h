// lbm_internal.h -- structures shared by the host runtime and the gfx950 kernels.
//
// Data layout in HBM (one cavity):
//   pop[2]  two population buffers (pull scheme: read one, write the other), each 19
//           planes: f0..f8, g0..g4, h0..h4.  A plane holds ny rows of `pitch` elements
//           (pitch >= nx, a multiple of 64), planes are `plane` elements apart
//           (plane >= ny*pitch, padded so that planes do not alias on the same HBM
//           channels).  Element (x, y) of plane i is at i*plane + y*pitch + x.
//   d4[2]   two buffers of 4 planes, the fields of the previous step: T - T0, C - C0, ux, uy
//           (FP64 for FP64 storage, FP32 otherwise).  The one-step kernel reads and rewrites the current
//           one in place (each node its own values); the multi-step kernels read one and write
//           the other (their halo nodes are read by neighbouring work-groups).
//   phi     1 plane of porosity (only when the porosity is a field).
//   snap    4 planes: residual snapshot of T - T0, C - C0, ux, uy.
//   counter 2 words: the step count, kept beside the state it belongs to (index = buffer).
//   Populations are stored as deviations from the rest state (rho0, T0, C0).
#pragma once
#include <stdint.h>

namespace lbmk {

enum { SIDE_HOT = 0, SIDE_COLD = 1, SIDE_ADIABATIC = 2, SIDE_PERIODIC = 3,
       SIDE_NEE_HOT = 4, SIDE_NEE_COLD = 5, SIDE_NEE_ADIABATIC = 6, SIDE_NEE_ROBIN = 7 };
enum { LEFT = 0, RIGHT = 1, BOTTOM = 2, TOP = 3 };
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP16S = 2 };
// cache policies of the step launch (see the kernels for what each sets)
enum { CP_TUNED = 0, CP_STREAM = 1, CP_RESIDENT = 2, CP_COUNT = 3 };
constexpr int NPOP = 19;       // 9 + 5 + 5 planes
constexpr int ND4 = 4;

// Per-cavity constants in the arithmetic type R of the kernel (double or float).
template <typename R>
struct Desc {
  int nx, ny, pitch, phi_field;
  long long plane;
  int perx, pery, ergun, model;
  int kind[4];
  int base_parity, pad_[3];
  void *pop0, *pop1;       // population buffers (storage type)
  void *d4;                // fields T - T0, C - C0, ux, uy of the current level (type R)
  void *d4b;               // the other field buffer (written by the two-step kernel)
  void *phi;               // porosity plane (type R), when phi_field
  unsigned *counter;       // step counters [2]: counter[cur] is the step count of the state in
                           // buffer cur (drives the FP16 stochastic rounding)
  R rho0, inv_rho0, sigma, inv_sigma, varpi, T0, C0;
  R s_e, s_eps, s_j, s_q, s_v;
  R z_a, z_e, z_eps, e_D, e_e, e_eps;
  R k_e, k_eps, k_j, k_q, k_v, k_za, k_eD;   // forcing weights 1 - s/2 of Eq. (10) and of the
                                             // D2Q5 source (Eq. 27) for the rates above
  R gbT, gbC, gx, gy;
  R phi_u, a_u, b_u;       // uniform porosity: phi, Darcy a = phi nu/K, Forchheimer b = phi F/sqrt(K)
  R ca, cb;                // porosity field: a = ca (1-phi)^2/phi^2; b = cb (1-phi)/phi^2 (Ergun)
                           // or cb (1-phi)/sqrt(phi) (fixed F_phi)
  R kg3, c5v;              // n3eq - n3ref = kg3 (T - T0) for g; c5v = 5 varpi
  R inv_phi_u, kh3_u;      // uniform porosity: 1/phi and the h energy factor (as kg3 for g)
  R wT[4], wC[4];          // anti-bounce-back constants (deviation form, pre-scaled) per side
  R uw[4];                 // 6 rho0 u_wall per side (moving-wall term of the bounce-back, pre-scaled)
  R uwall[4];              // tangential wall velocity per side
  R scale, inv_scale;      // FP16 pre-scale (1 for FP32/FP64)
  R rho0_s, inv_rho0_s;    // rho0 scale and 1/(rho0 scale): the collision's constants in the units
  R T0_s, C0_s;            // of the pre-scale (T0 scale, C0 scale; unscaled for FP32/FP64)
  // walls through the boundary nodes (side kinds 4-7)
  int nee, pad2_[3];
  R Tfix[4], Cfix[4];      // fixed T - T0, C - C0 of each side (kinds 4, 5)
  R betaT[4], betaC[4];    // Bi/L of each side (kind 7), 0 otherwise
  R Tinf, Cinf;            // ambient of a convective side, as T - T0, C - C0
  R kg0, capT, capC;       // g0 equilibrium factor and the T, C capacities of g_i^eq, h_i^eq
};

struct Item {              // one tile of one cavity, for the batched kernel: tw nodes along x
  int cavity, x0, y0, tw;  // (64, 128 or 256) by 256/tw rows, one node per thread
};

// Launch shape of the step kernel
struct Tile {
  int tx, ty;
};

// ---- launchers (defined in lbm_kernels.hip) ---------------------------------------------
// All take a hipStream_t as void*; return a hipError_t as int.
int launch_init(int prec, const void *desc, const double *T, const double *C, const double *ux,
                const double *uy, void *stream);
// desc: the host copy of the descriptor (launch geometry); ddev: the same descriptor in device
// memory, which the step kernels read.  cp: cache policy CP_*
int launch_step(int prec, const void *desc, const void *ddev, Tile tile, int cp, int parity, void *stream);
// two time steps per launch (tiles with a one-node halo staged in LDS); fields read from d4,
// written to d4b; walls through the nodes with FP32 and FP64 storage on lattices of at least
// one tile (else hipErrorInvalidValue).  sw: tile order, row by row (0) or in vertical strips of
// sw tiles; rows: tile rows, 8 (64 x 8, FP64 32 x 8) or, FP16 storage without node walls only,
// 12 (64 x 12); else hipErrorInvalidValue
int launch_step2(int prec, const void *desc, const void *ddev, int cp, int parity, int sw, int rows, void *stream);
// three time steps per launch (tiles with a two-node halo staged in LDS); FP32 and FP64
// storage, walls half a spacing outside; fields read from d4, written to d4b; sw as above;
// rows: tile rows, 8 (64 x 8, FP64 32 x 8) or, FP32 only, 12 (64 x 12); else hipErrorInvalidValue
int launch_step3(int prec, const void *desc, const void *ddev, int cp, int parity, int sw, int rows, void *stream);
// range: device pointer to {first item, item count} of the group to step; parity bit 0
// selects the population buffers, bit 1 the field buffer (d4b when set)
int launch_step_batch(int prec, int cp, const void *descs, const Item *items, const int *range, int grid, int parity,
                      void *stream);
// two steps per launch over items of two-step tiles of shape `shape` (0 .. batch_tile_shapes()-1;
// item.tw = tile width), one item per work-group: grid >= the group's item count; parity as
// above for both the population and the field buffers
int launch_step2_batch(int prec, int cp, int shape, const void *descs, const Item *items, const int *range, int grid,
                       int parity, void *stream);
// three steps per launch over the items of batch tile shape 0 (the three-step tile), one item
// per work-group; FP32 and FP64 storage only (else hipErrorInvalidValue); parity as above
int launch_step3_batch(int prec, int cp, const void *descs, const Item *items, const int *range, int grid,
                       int parity, void *stream);
// two steps per launch with walls through the boundary nodes over items of two-step tiles
// (shape 0) placed against the far walls as the single-cavity two-step kernel places its last
// tiles; FP32 and FP64 only (else hipErrorInvalidValue); parity as above
int launch_step2_batch_nee(int prec, int cp, const void *descs, const Item *items, const int *range, int grid,
                           int parity, void *stream);
// tile of the single-cavity two-step kernels for a storage precision
void two_step_tile_shape(int prec, int *w, int *h);
// tile shapes of the batched two-step kernel
int batch_tile_shapes();
void batch_tile_shape(int prec, int shape, int *w, int *h);
// observables: partial sums per block, then a final fixed-order reduction.
// out: 16 doubles + Nu[4] + Sh[4] (see lbm_api.cpp for the slots)
int launch_observables(int prec, const void *desc, int parity, void *snap, double *partials,
                       int nblocks, double *out, const double *wall_T, const double *wall_C,
                       double L_over_dT, double L_over_dC, void *stream);
int launch_export(int prec, const void *desc, int parity, double *fields, void *stream);
int observables_blocks(int ny);

// Fixed device scratch of the no-allocation observables (offsets in doubles)
struct StaticScratchLayout {
  int max_rows;              // tallest lattice whose observables partials fit
  long long max_nodes;       // largest lattice whose exported fields fit
  long long out, partials, fields, doubles;
};
StaticScratchLayout static_scratch_layout();
// device address of the scratch array on `device`, which must be current (looked up once per
// device); hipError_t as int
int static_scratch_address(int device, double **ptr);

}  // namespace lbmk
