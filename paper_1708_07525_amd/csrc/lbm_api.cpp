// lbm_api.cpp -- host runtime behind the C ABI of include/lbm.h: parameter mapping and
// validation (sections 2 and 4.1, Eq. 29), device buffers, launch bookkeeping, HIP graph
// replay of step chunks, reductions, checkpoints, the autotuner and the batch table.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

namespace {
// a roctx range around each entry point that does device work, so that a profiler run
// (rocprofv3 --marker-trace) shows steps, observables and tuning on the host timeline
struct Range {
  explicit Range(const char *name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};
}  // namespace

#define LBM_API extern "C" __attribute__((visibility("default")))

using namespace lbmk;

namespace {

constexpr int kGraphChunk = 64;     // default steps per captured graph in lbm_step (even)
constexpr double kCs2 = 1.0 / 3.0;  // D2Q9 sound speed squared

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// element sizes
size_t store_size(int prec) { return prec == PREC_FP64 ? 8 : (prec == PREC_FP32 ? 4 : 2); }
size_t real_size(int prec) { return prec == PREC_FP64 ? 8 : 4; }

struct Layout {
  int pitch;
  long long plane;
  size_t off_pop0, off_pop1, off_d4, off_d4b, off_phi, off_snap, off_counter, off_desc, off_small, total;
  int nblocks_obs;
};

// device copies of the descriptor, one per (population buffer, field buffer) of a launch
constexpr size_t kDescSlot = 1024;
static_assert(sizeof(Desc<double>) <= kDescSlot && sizeof(Desc<float>) <= kDescSlot, "descriptor slot");

// Planes of ny rows of `pitch` elements; the plane stride is padded by 256 elements past a
// 1024-element boundary so that the 19 + 4 concurrent streams do not start on the same
// HBM channel.
constexpr double kMaxResourceBytes = 4294967295.0;   // largest range of one buffer resource

Layout plan_layout(int nx, int ny, int prec) {
  Layout L{};
  const size_t es = store_size(prec), rs = real_size(prec);
  L.pitch = (int)round_up((size_t)nx, 64);
  L.plane = (long long)round_up((size_t)L.pitch * ny, 1024) + 256;
  L.nblocks_obs = observables_blocks(ny);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = round_up(off + bytes, 4096);
    return o;
  };
  L.off_pop0 = take((size_t)NPOP * L.plane * es);
  L.off_pop1 = take((size_t)NPOP * L.plane * es);
  L.off_d4 = take((size_t)ND4 * L.plane * rs);
  L.off_d4b = take((size_t)ND4 * L.plane * rs);   // second field buffer of the multi-step launches
  L.off_phi = take((size_t)L.plane * rs);
  L.off_snap = take((size_t)ND4 * L.plane * rs);
  L.off_counter = take(2 * sizeof(unsigned));
  L.off_desc = take(4 * kDescSlot);
  // small: wall T (4), wall C (4), obs out (32), partials
  L.off_small = take((8 + 32 + (size_t)L.nblocks_obs * 12) * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

struct lbm_ctx {
  lbm_params p{};
  Layout lay{};
  int prec = PREC_FP32;
  hipStream_t stream = nullptr;
  int device = 0;
  char *base = nullptr;      // device memory (arena or owned)
  bool owned = false;
  bool ready = false;
  bool unstable = false;     // lbm_observables found a non-finite value: lbm_step refuses to go on
  double *scratch = nullptr; // device address of the fixed scratch on this context's device
  lbm_batch *batch = nullptr;   // the batch this context is attached to, if any
  int cur = 0;               // buffer holding the post-collision state of the current level
  int d4cur = 0;             // field buffer (d4 or d4b) holding the fields of the current level
  int steps_per_launch = 0;  // 1, 2, or 0: chosen by the default rule
  int64_t step = 0;
  int64_t snap_step = 0;
  Tile tile{256, 1};
  int cache_policy = -1;     // CP_* or -1: chosen by the bytes a step touches
  int strip = -1;            // tile order of the multi-step launches (strip width), -1: default_strip
  int tile_rows = 0;         // rows of the FP32 three-step / FP16 two-step tile, 0: default_rows
  lbm_derived dv{};
  bool phi_field = false;
  Desc<double> d64{};
  Desc<float> d32{};
  double wallT[4]{}, wallC[4]{};   // wall T and C minus T0, C0, per side
  std::string err;
  // graph of kGraphChunk steps, valid for `graph_cur` and `graph_tile`
  hipGraphExec_t graph = nullptr;
  int graph_cur = -1;
  Tile graph_tile{0, 0};
  int graph_cp = -1;
  int graph_d4 = -1, graph_spl = 0, graph_sw = -1, graph_rows = 0;
  int graph_chunk = kGraphChunk;   // 0: plain launches only

  void *pop(int i) const { return base + (i ? lay.off_pop1 : lay.off_pop0); }
  void *d4() const { return base + (d4cur ? lay.off_d4b : lay.off_d4); }
  void *d4other() const { return base + (d4cur ? lay.off_d4 : lay.off_d4b); }
  void *phi() const { return base + lay.off_phi; }
  void *snap() const { return base + lay.off_snap; }
  unsigned *counter() const { return (unsigned *)(base + lay.off_counter); }
  double *wall_dev() const { return (double *)(base + lay.off_small); }
  double *obs_out() const { return wall_dev() + 8; }
  double *partials() const { return wall_dev() + 40; }
  const void *desc() const { return prec == PREC_FP64 ? (const void *)&d64 : (const void *)&d32; }
  // the device copy of the descriptor for population buffer `pc` and field buffer `fc`
  const void *desc_dev(int pc, int fc) const { return base + lay.off_desc + (size_t)(2 * pc + fc) * kDescSlot; }
};

namespace {

lbm_status fail(lbm_ctx *c, lbm_status s, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

lbm_status hip_fail(lbm_ctx *c, hipError_t e, const char *what) {
  return fail(c, LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_CHECK(ctx, expr, what)                 \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

bool rate_ok(double s) { return s > 0.0 && s < 2.0; }

// Validation of everything that does not need the porosity field.
lbm_status validate(const lbm_params *p, std::string &msg) {
  auto bad = [&](const char *m) {
    msg = m;
    return LBM_EINVAL;
  };
  if (p->nx < 3 || p->ny < 3) return bad("nx and ny must be >= 3");
  if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return bad("lattice too large");
  if (p->precision < 0 || p->precision > 2) return bad("unknown precision");
  // the kernels address the 19 population planes of a buffer through one buffer resource with
  // 32-bit byte offsets
  if ((double)NPOP * (double)plan_layout(p->nx, p->ny, p->precision).plane * (double)store_size(p->precision) >
      kMaxResourceBytes)
    return bad("lattice too large for this storage type: the 19 population planes of a buffer must fit "
               "in 4 GiB (about 28M nodes in FP64, 56M in FP32, 113M in FP16)");
  if (p->model != 0 && p->model != 1) return bad("model must be 0 (present) or 1 (Model-A)");
  int n_half = 0, n_node = 0;
  for (int s = 0; s < 4; ++s) {
    if (p->side[s] < 0 || p->side[s] > 7) return bad("unknown side kind");
    if (p->side[s] <= SIDE_ADIABATIC) n_half++;
    if (p->side[s] >= SIDE_NEE_HOT) n_node++;
  }
  if (n_half && n_node) return bad("walls half a spacing outside and walls through the nodes cannot be mixed");
  if (n_node && p->side[LEFT] != SIDE_PERIODIC && p->nx < 5) return bad("walls through the nodes need nx >= 5");
  if (n_node && p->side[BOTTOM] != SIDE_PERIODIC && p->ny < 5) return bad("walls through the nodes need ny >= 5");
  if (!(p->Bi_T >= 0.0) || !(p->Bi_C >= 0.0)) return bad("Biot numbers must be >= 0");
  if ((p->side[LEFT] == SIDE_PERIODIC) != (p->side[RIGHT] == SIDE_PERIODIC) ||
      (p->side[BOTTOM] == SIDE_PERIODIC) != (p->side[TOP] == SIDE_PERIODIC))
    return bad("periodic sides must come in opposite pairs");
  if (!(p->phi > 0.0 && p->phi <= 1.0)) return bad("porosity must lie in (0, 1]");
  if (!(p->sigma > 0.0) || !(p->J > 0.0) || !(p->rho0 > 0.0)) return bad("sigma, J and rho0 must be positive");
  if (p->varpi >= 1.0) return bad("varpi must lie in (0, 1)");
  const double rates[] = {p->s_rho, p->s_e, p->s_eps, p->s_j, p->s_q, p->zeta0, p->zeta_e, p->zeta_eps,
                          p->eta0, p->eta_e, p->eta_eps};
  for (double r : rates)
    if (!rate_ok(r)) return bad("free relaxation rates must lie in (0, 2)");
  if (p->direct < 0 || p->direct > 2) return bad("direct must be 0 (natural convection), 1 (lattice values) or 2 "
                                                  "(lid-driven mixed convection)");
  if (p->direct == 2) {
    if (!(p->Re > 0) || !(p->Gr >= 0) || !(p->U0 > 0) || !(p->Pr > 0) || !(p->Le > 0) || !(p->Da > 0))
      return bad("Re, U0, Pr, Le and Da must be positive and Gr >= 0");
    if (!(p->Th - p->Tl > 0) || !(p->Ch - p->Cl > 0)) return bad("Th > Tl and Ch > Cl are required");
  } else if (p->direct) {
    if (!(p->nu > 0) || !(p->alpha_e > 0) || !(p->D_e > 0) || !(p->K > 0))
      return bad("direct lattice values nu, alpha_e, D_e, K must be positive");
  } else {
    if (!(p->Ra > 0) || !(p->Pr > 0) || !(p->Le > 0) || !(p->Da > 0) || !(p->Ma > 0))
      return bad("Ra, Pr, Le, Da and Ma must be positive");
    if (!(p->Th - p->Tl > 0) || !(p->Ch - p->Cl > 0)) return bad("Th > Tl and Ch > Cl are required");
  }
  return LBM_OK;
}

// Lattice values of sections 2 and 4.1 (nothing that needs the porosity field).
bool node_walls(const lbm_params *p) {
  for (int s = 0; s < 4; ++s)
    if (p->side[s] >= SIDE_NEE_HOT) return true;
  return false;
}

// Default launch shape: one row of 256, 128 or 64 nodes, whichever wastes the fewest lanes
// on the ragged right edge of the columns the tiles cover (ties go to the wider tile); with
// walls through the nodes the last column belongs to the perimeter work.
Tile default_tile(const lbm_params *p) {
  const int w = p->nx - (node_walls(p) && p->side[LEFT] != SIDE_PERIODIC ? 1 : 0);
  int tw = 256;
  for (int cand : {128, 64})
    if ((w + cand - 1) / cand * cand < (w + tw - 1) / tw * tw) tw = cand;
  return Tile{tw, 1};
}

// algorithmic bytes of one node update (19 population loads and stores, 4 + 4 field
// accesses, 1 porosity load)
double bytes_per_lu(int prec) { return prec == PREC_FP64 ? 376.0 : (prec == PREC_FP32 ? 188.0 : 112.0); }

// Steps per launch when none is set: three for FP32 and FP64 storage (faster than two at every
// lattice size measured, 256^2 to 4096^2: 2048^2 FP32 60.6 against 49.7 GLUPS, FP64 27.1
// against 24.2), two for FP16 storage (held by its arithmetic, to which a third step would add
// a sixth); where a count does not apply the next lower one is taken (two_step_ok,
// three_step_ok).
int default_spl(int prec, double nodes) {
  (void)nodes;
  return prec == PREC_FP16S ? 2 : 3;
}

// Cache policy when none is set: a step that touches at most 400 MB keeps its data in the
// 256 MB Infinity Cache between steps for the most part, so plain loads and stores win
// (CP_RESIDENT); above that the multi-step kernels stream with non-temporal stores
// (CP_STREAM), and so does the one-step FP32 kernel, while the one-step FP16 and FP64
// kernels keep their tuned policy (measured on 512^2 to 4096^2 lattices).
int default_policy(int prec, double nodes, int spl) {
  if (nodes * bytes_per_lu(prec) <= 400e6) return CP_RESIDENT;
  return (spl >= 2 || prec == PREC_FP32) ? CP_STREAM : CP_TUNED;
}

// Tile order of the multi-step launches when none is set (lbm_set_strip_width): vertical strips
// of sw tiles.  Row by row, a tile's halo rows were loaded a whole row of tiles earlier and have
// left the L2 on wide lattices; in strips they were loaded sw tiles earlier.  The strips pay most
// when they line up with the 8 XCD bands of the launch (an XCD's band is a whole number of
// strips, or the reverse): FP32 three steps per launch on 64 x 12 tiles, 1536^2 (24 tiles across)
// 63.9 GLUPS with strips of 3 against 58.8 with 4 and 62.2 row by row; 2560^2 (40) 69.7 with 5
// against 65.9 with 8; 3072^2 (48) 72.0 with 6 against 67.4 with 8; 2048^2 (32) 67.3 with 4;
// 4096^2 (64) 73.2 with 8; FP16 two steps on 64 x 12 tiles 2560^2 72.5 with 5 against 69.2 with 8,
// 3072^2 74.7 with 6.  Narrow strips of 2 lose to their edge columns (2048^2, 64 x 8: 55.2), and
// where the tiles across are not a multiple of 8, strips of 8 come within 2% of the best width
// while 4 loses up to 8% (1800^2 FP32 62.5 with 8, 56.9 with 4; 1900^2 FP16 67.0 against 61.6;
// 2600 x 1600 63.9 against 57.7, best 65.1 with 7).  Rule for the three-step launches and the
// two-step ones on 12-row tiles: ntx/8 tiles when the tiles across are a multiple of 8 (halved
// while above 8), else 8.
// Two-step launches on 64 x 8 tiles (walls through the nodes) lose with strips at 2048^2 (48.7 row
// by row, 43.3 with 4, 46.6 with 8) and gain at 4096^2 (52.2 with 8 against 47.6): row by row up
// to 32 tiles across, 8 beyond.  Lattices that stay in the Infinity Cache (at most 400 MB per
// step) go row by row (1024^2, 64 x 8: 65.0 against 62.9-64.4 with strips).
int default_strip(int prec, int nx, int ny, int spl, int rows) {
  if (spl < 2) return 0;
  int w = 0, h = 0;
  two_step_tile_shape(prec, &w, &h);
  const int ntx = (nx + w - 1) / w;
  if (ntx <= 8 || (double)nx * ny * bytes_per_lu(prec) <= 400e6) return 0;
  if (spl == 2 && rows != 12) return ntx > 32 ? 8 : 0;
  if (ntx % 8 == 0) {
    int a = ntx / 8;
    while (a > 8 && a % 2 == 0) a /= 2;
    if (a >= 3 && a <= 16) return a;
  }
  return 8;
}

// Rows of the multi-step tile when none is set (lbm_set_tile_rows): the FP32 three-step and the
// FP16 two-step launch take the 64 x 12 tile where a step touches more than 400 MB (the lattice
// streams from HBM: FP32 2048^2 67.3 against 62.9 GLUPS for 64 x 8, 4096^2 74.4 against 68.6;
// FP16 2048^2 69.5 against 67.3, 4096^2 76.2 against 71.9) and 64 x 8 below (the lattice stays in
// the Infinity Cache, where the third work-group per CU of the smaller tile wins: FP32 1024^2 65.0
// against 61.1); FP64 and the node-wall launches have the 8-row tile only.
int default_rows(int prec, double nodes) {
  return (prec != PREC_FP64 && nodes * bytes_per_lu(prec) > 400e6) ? 12 : 8;
}

void map_params(const lbm_params *p, lbm_derived &d) {
  // cavity width: nx for walls half a spacing outside, nx - 1 for walls through the nodes
  d.L = node_walls(p) ? p->nx - 1 : p->nx;
  d.dT = p->Th - p->Tl;
  d.T0 = 0.5 * (p->Th + p->Tl);
  d.dC = p->Ch - p->Cl;
  d.C0 = 0.5 * (p->Ch + p->Cl);
  if (p->direct == 2) {
    // section 4.3, mixed convection in a lid-driven cavity: Re = U0 L/nu, i.e.
    // 1/s_v = 1/2 + J L U0/(c_s^2 Re); Gr = g beta_T dT L^3/nu^2; Pr, Le, Da, N as above
    d.U = p->U0;
    d.nu = p->U0 * d.L / p->Re;
    d.alpha_e = d.nu / p->Pr;
    d.D_e = d.alpha_e / p->Le;
    d.K_mean = p->Da * d.L * d.L;
    d.gbT = p->Gr * d.nu * d.nu / (d.L * d.L * d.L * d.dT);
    d.gbC = p->N * d.gbT * d.dT / d.dC;
  } else if (p->direct) {
    d.nu = p->nu;
    d.alpha_e = p->alpha_e;
    d.D_e = p->D_e;
    d.K_mean = p->K;
    d.gbT = p->gbT;
    d.gbC = p->gbC;
    d.U = std::sqrt(std::fabs(d.gbT * d.dT * d.L));
  } else {
    // Ma = U/c_s; U^2 = g beta_T dT L; Ra = g beta_T dT L^3/(nu alpha_e); Pr = nu/alpha_e
    d.U = p->Ma * std::sqrt(kCs2);
    d.nu = d.U * d.L * std::sqrt(p->Pr / p->Ra);
    d.alpha_e = d.nu / p->Pr;
    d.D_e = d.alpha_e / p->Le;
    d.K_mean = p->Da * d.L * d.L;
    d.gbT = d.U * d.U / (d.L * d.dT);
    d.gbC = p->N * d.gbT * d.dT / d.dC;
  }
  d.nu_e = p->J * d.nu;
  d.s_v = 1.0 / (0.5 + d.nu_e / kCs2);
}

// The relaxation rates and model parameter that need varpi, known once the smallest porosity
// is: Eq. (29) (present model) or Eq. (32) (Model-A) with c_sT^2 = varpi/2; and the FP16
// pre-scale.  Returns a message on an out-of-range rate.
const char *derive_rates(const lbm_params *p, int prec, double phi_min, lbm_derived &d) {
  d.phi_min = phi_min;
  d.varpi = p->varpi > 0 ? p->varpi : std::min(0.4, phi_min);
  d.csT2 = 0.5 * d.varpi;
  if (p->model == 0) {
    d.zeta_a = 1.0 / (0.5 + d.alpha_e / d.csT2);  // Eq. (29)
    d.eta_D = 1.0 / (0.5 + d.D_e / d.csT2);
  } else {
    d.zeta_a = 1.0 / (0.5 + d.alpha_e / (p->sigma * d.csT2));  // Eq. (32)
    d.eta_D = 1.0 / (0.5 + d.D_e / (p->phi * d.csT2));
  }
  // FP16 pre-scale: a power of two that keeps deviations of size up to 16x the wall
  // contrast inside the binary16 range
  double B = 0.5;
  B = std::max(B, std::max(p->sigma, 1.0) * std::max(std::fabs(p->Th - d.T0), std::fabs(p->Tl - d.T0)));
  B = std::max(B, std::max(std::fabs(p->Ch - d.C0), std::fabs(p->Cl - d.C0)));
  d.fp16_scale = prec == PREC_FP16S ? std::ldexp(1.0, (int)std::floor(std::log2(4096.0 / B))) : 1.0;
  if (!rate_ok(d.s_v)) return "derived s_v outside (0, 2)";
  if (!rate_ok(d.zeta_a)) return "derived zeta_alpha outside (0, 2)";
  if (!rate_ok(d.eta_D)) return "derived eta_D outside (0, 2)";
  return nullptr;
}

// Everything that needs varpi (known once the porosity field is).
lbm_status finish_mapping(lbm_ctx *c, double phi_min, double mean_kc) {
  const lbm_params *p = &c->p;
  lbm_derived &d = c->dv;
  if (const char *m = derive_rates(p, c->prec, phi_min, d))
    return fail(c, LBM_EINVAL, "%s (s_v = %g, zeta_alpha = %g, eta_D = %g)", m, d.s_v, d.zeta_a, d.eta_D);
  if (p->varpi > phi_min)
    c->err = "note: varpi exceeds the smallest porosity; the concentration scheme may be unstable";

  // fill both descriptor types from FP64 values
  auto fill = [&](auto &D) {
    using R = std::remove_reference_t<decltype(D.rho0)>;
    D = {};
    D.nx = p->nx;
    D.ny = p->ny;
    D.pitch = c->lay.pitch;
    D.plane = c->lay.plane;
    D.perx = p->side[LEFT] == SIDE_PERIODIC;
    D.pery = p->side[BOTTOM] == SIDE_PERIODIC;
    D.phi_field = c->phi_field;
    D.ergun = p->Fphi < 0;
    D.model = p->model;
    for (int s = 0; s < 4; ++s) D.kind[s] = p->side[s];
    D.base_parity = 0;
    D.pop0 = c->pop(0);
    D.pop1 = c->pop(1);
    D.d4 = c->d4();
    D.d4b = c->d4other();
    D.phi = c->phi();
    D.counter = c->counter();
    D.rho0 = (R)p->rho0;
    D.inv_rho0 = (R)(1.0 / p->rho0);
    D.sigma = (R)p->sigma;
    D.inv_sigma = (R)(1.0 / p->sigma);
    D.varpi = (R)d.varpi;
    D.T0 = (R)d.T0;
    D.C0 = (R)d.C0;
    D.s_e = (R)p->s_e;
    D.s_eps = (R)p->s_eps;
    D.s_j = (R)p->s_j;
    D.s_q = (R)p->s_q;
    D.s_v = (R)d.s_v;
    D.z_a = (R)d.zeta_a;
    D.z_e = (R)p->zeta_e;
    D.z_eps = (R)p->zeta_eps;
    D.e_D = (R)d.eta_D;
    D.e_e = (R)p->eta_e;
    D.e_eps = (R)p->eta_eps;
    D.k_e = R(1) - R(0.5) * D.s_e;
    D.k_eps = R(1) - R(0.5) * D.s_eps;
    D.k_j = R(1) - R(0.5) * D.s_j;
    D.k_q = R(1) - R(0.5) * D.s_q;
    D.k_v = R(1) - R(0.5) * D.s_v;
    D.k_za = R(1) - R(0.5) * D.z_a;
    D.k_eD = R(1) - R(0.5) * D.e_D;
    D.gbT = (R)d.gbT;
    D.gbC = (R)d.gbC;
    D.gx = (R)p->g_ext[0];
    D.gy = (R)p->g_ext[1];
    // uniform porosity: a = phi nu/K, b = phi F_phi/sqrt(K) (Eq. 5), K = Da L^2
    const double phi = p->phi;
    const double F = p->Fphi >= 0 ? p->Fphi : 1.75 / std::sqrt(150.0 * phi * phi * phi);  // Eq. (7)
    D.phi_u = (R)phi;
    D.a_u = (R)(phi * d.nu / d.K_mean);
    D.b_u = (R)(phi * F / std::sqrt(d.K_mean));
    // porosity field: K(x) = Ks phi^3/(1-phi)^2 with Ks = K_mean / mean(phi^3/(1-phi)^2)
    const double Ks = mean_kc > 0 ? d.K_mean / mean_kc : d.K_mean;
    D.ca = (R)(d.nu / Ks);
    D.cb = (R)(p->Fphi < 0 ? 1.75 / std::sqrt(150.0 * Ks) : p->Fphi / std::sqrt(Ks));
    D.kg3 = (R)(p->model == 0 ? 5.0 * d.varpi - 4.0 * p->sigma : (5.0 * d.varpi - 4.0) * p->sigma);
    D.c5v = (R)(5.0 * d.varpi);
    D.inv_phi_u = (R)(1.0 / phi);
    D.kh3_u = (R)(p->model == 0 ? 5.0 * d.varpi - 4.0 * phi : (5.0 * d.varpi - 4.0) * phi);
    const double capT = p->model == 0 ? 1.0 : p->sigma;
    const double capC = p->model == 0 ? 1.0 : p->phi;
    for (int s = 0; s < 4; ++s) {
      const double Tw = p->side[s] == SIDE_HOT ? p->Th : p->Tl;
      const double Cw = p->side[s] == SIDE_HOT ? p->Ch : p->Cl;
      // anti-bounce-back: g_i = -g*_opp + g^eq_i(w) + g^eq_opp(w) = -g*_opp + (varpi/2) cap T_w,
      // in deviation form -gd*_opp + (varpi/2) cap (T_w - T0)
      // (in the units of the FP16 pre-scale, as the populations they are added to)
      D.wT[s] = (R)(0.5 * d.varpi * capT * (Tw - d.T0) * d.fp16_scale);
      D.wC[s] = (R)(0.5 * d.varpi * capC * (Cw - d.C0) * d.fp16_scale);
      D.uw[s] = (R)(6.0 * p->rho0 * p->wall_u[s] * d.fp16_scale);
      D.uwall[s] = (R)p->wall_u[s];
    }
    D.scale = (R)d.fp16_scale;
    D.inv_scale = (R)(1.0 / d.fp16_scale);
    D.rho0_s = (R)(p->rho0 * d.fp16_scale);
    D.inv_rho0_s = (R)(1.0 / (p->rho0 * d.fp16_scale));
    D.T0_s = (R)(d.T0 * d.fp16_scale);
    D.C0_s = (R)(d.C0 * d.fp16_scale);
    D.nee = node_walls(p);
    for (int s = 0; s < 4; ++s) {
      const bool hot = p->side[s] == SIDE_NEE_HOT;
      D.Tfix[s] = (R)((hot ? p->Th : p->Tl) - d.T0);
      D.Cfix[s] = (R)((hot ? p->Ch : p->Cl) - d.C0);
      D.betaT[s] = (R)(p->side[s] == SIDE_NEE_ROBIN ? p->Bi_T / d.L : 0.0);
      D.betaC[s] = (R)(p->side[s] == SIDE_NEE_ROBIN ? p->Bi_C / d.L : 0.0);
    }
    D.Tinf = (R)(p->Tl - d.T0);
    D.Cinf = (R)(p->Cl - d.C0);
    D.kg0 = (R)(p->model == 0 ? p->sigma - d.varpi : (1.0 - d.varpi) * p->sigma);
    D.capT = (R)capT;
    D.capC = (R)capC;
  };
  fill(c->d64);
  fill(c->d32);
  for (int s = 0; s < 4; ++s) {
    const bool hot = p->side[s] == SIDE_HOT || p->side[s] == SIDE_NEE_HOT;
    // wall values minus T0, C0: the wall-gradient stencils act on the stored deviations
    c->wallT[s] = (hot ? p->Th : p->Tl) - d.T0;
    c->wallC[s] = (hot ? p->Ch : p->Cl) - d.C0;
  }
  return LBM_OK;
}

// descriptor state for a launch that starts from population buffer `cur` and field buffer
// `d4cur` (the context's own, unless a graph capture is simulating later launches)
void set_parity(lbm_ctx *c, int cur, int d4cur) {
  c->d64.base_parity = cur;
  c->d32.base_parity = cur;
  void *fa = c->base + (d4cur ? c->lay.off_d4b : c->lay.off_d4);
  void *fb = c->base + (d4cur ? c->lay.off_d4 : c->lay.off_d4b);
  c->d64.d4 = fa;
  c->d32.d4 = fa;
  c->d64.d4b = fb;
  c->d32.d4b = fb;
}
void set_parity(lbm_ctx *c, int cur) { set_parity(c, cur, c->d4cur); }

bool arch_ok(int dev, std::string &name) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  name = prop.gcnArchName;
  return name.rfind("gfx950", 0) == 0;
}

void drop_graph(lbm_ctx *c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  c->graph_cur = -1;
}

}  // namespace

// ================================================================== C ABI

LBM_API void lbm_params_default(lbm_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->nx = p->ny = 64;
  p->precision = LBM_FP32;
  p->model = 0;
  p->side[LEFT] = LBM_SIDE_HOT;
  p->side[RIGHT] = LBM_SIDE_COLD;
  p->side[BOTTOM] = LBM_SIDE_ADIABATIC;
  p->side[TOP] = LBM_SIDE_ADIABATIC;
  p->Ra = 1e4;
  p->Pr = 1.0;
  p->Le = 2.0;
  p->Da = 1e-2;
  p->N = 1.0;
  p->J = 1.0;
  p->sigma = 1.0;
  p->phi = 0.6;
  p->Ma = 0.1;
  p->varpi = 0.0;
  p->rho0 = 1.0;
  p->s_rho = 1.0;
  p->s_e = 1.1;
  p->s_eps = 1.1;
  p->s_j = 1.0;
  p->s_q = 1.2;
  p->zeta0 = p->eta0 = 1.0;
  p->zeta_e = p->zeta_eps = p->eta_e = p->eta_eps = 1.5;
  p->Th = 1.0;
  p->Tl = 0.0;
  p->Ch = 1.0;
  p->Cl = 0.0;
  p->Fphi = -1.0;
}

LBM_API uint64_t lbm_footprint_bytes(const lbm_params *p) {
  if (!p || p->nx < 3 || p->ny < 3 || p->precision < 0 || p->precision > 2) return 0;
  return plan_layout(p->nx, p->ny, p->precision).total;
}

LBM_API lbm_status lbm_derive(const lbm_params *p, lbm_derived *out) {
  if (!p || !out) return LBM_EINVAL;
  std::string msg;
  if (validate(p, msg) != LBM_OK) return LBM_EINVAL;
  lbm_derived d{};
  map_params(p, d);
  if (derive_rates(p, p->precision, p->phi, d)) return LBM_EINVAL;
  *out = d;
  return LBM_OK;
}

LBM_API lbm_status lbm_create(const lbm_params *p, lbm_ctx **out) {
  if (!p || !out) return LBM_EINVAL;
  std::string msg;
  lbm_status s = validate(p, msg);
  if (s != LBM_OK) return s;
  lbm_ctx *c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ENOMEM;
  c->p = *p;
  c->prec = p->precision;
  c->stream = (hipStream_t)p->stream;
  c->lay = plan_layout(p->nx, p->ny, p->precision);
  map_params(p, c->dv);
  c->tile = default_tile(p);
  std::string arch;
  if (hipGetDevice(&c->device) != hipSuccess || !arch_ok(c->device, arch)) {
    delete c;
    return LBM_EDEVICE;
  }
  // the fixed scratch of lbm_observables_static: its address on this (current) device
  if (static_scratch_address(c->device, &c->scratch) != (int)hipSuccess) {
    delete c;
    return LBM_EDEVICE;
  }
  if (p->arena) {
    if (p->arena_bytes < c->lay.total || ((uintptr_t)p->arena & 255)) {
      delete c;
      return LBM_ENOMEM;
    }
    c->base = (char *)p->arena;
  } else {
    if (hipMalloc((void **)&c->base, c->lay.total) != hipSuccess) {
      delete c;
      return LBM_ENOMEM;
    }
    c->owned = true;
  }
  *out = c;
  return LBM_OK;
}

static void batch_forget(lbm_batch *b, lbm_ctx *c);

LBM_API void lbm_destroy(lbm_ctx *c) {
  if (!c) return;
  if (c->batch) {
    // still attached: the batch forgets it once the work queued on the batch stream is done,
    // so no later replay reaches the memory freed here
    lbm_batch *b = c->batch;
    if (lbm_batch_detach(b, c) != LBM_OK) {
      (void)hipStreamSynchronize(c->stream);
      batch_forget(b, c);
    }
  }
  drop_graph(c);
  if (c->owned && c->base) (void)hipFree(c->base);
  delete c;
}

LBM_API const char *lbm_last_error(const lbm_ctx *c) {
  if (!c) return "no context";
  return c->err.c_str();
}

LBM_API lbm_status lbm_set_fields(lbm_ctx *c, const double *phi, const double *T, const double *C,
                                  const double *ux, const double *uy) {
  Range range_("lbm_set_fields");
  if (!c) return LBM_EINVAL;
  if (c->batch) return fail(c, LBM_ESTATE, "context is attached to a batch");
  c->err.clear();
  const lbm_params *p = &c->p;
  const size_t n = (size_t)p->nx * p->ny;
  // porosity: validation, smallest value and the Kozeny-Carman mean
  double phi_min = p->phi, mean_kc = 0.0;
  c->phi_field = phi != nullptr;
  if (phi) {
    if (p->model == 1) return fail(c, LBM_EINVAL, "Model-A needs a uniform porosity");
    phi_min = 1e300;
    double s = 0.0;
    for (size_t k = 0; k < n; ++k) {
      const double q = phi[k];
      if (!(q > 0.0 && q < 1.0)) return fail(c, LBM_EINVAL, "porosity field values must lie in (0, 1)");
      phi_min = std::min(phi_min, q);
      s += q * q * q / ((1.0 - q) * (1.0 - q));
    }
    mean_kc = s / (double)n;
  }
  lbm_status st = finish_mapping(c, phi_min, mean_kc);
  if (st != LBM_OK) return st;
  drop_graph(c);
  c->cur = 0;
  c->d4cur = 0;
  set_parity(c, 0);
  // stage the inputs (FP64) on the device
  const size_t plane_bytes = (size_t)c->lay.plane * real_size(c->prec);
  double *stage = nullptr;
  HIP_CHECK(c, hipMalloc((void **)&stage, 4 * n * sizeof(double)), "hipMalloc staging");
  std::vector<double> fill;
  auto put = [&](const double *src, double def, int slot) -> hipError_t {
    if (!src) {
      fill.assign(n, def);
      src = fill.data();
    }
    return hipMemcpyAsync(stage + slot * n, src, n * sizeof(double), hipMemcpyHostToDevice, c->stream);
  };
  hipError_t e = put(T, c->dv.T0, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = put(C, c->dv.C0, 1);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = put(ux, 0.0, 2);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = put(uy, 0.0, 3);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  // every buffer starts zeroed, row and plane padding included, so that checkpoints
  // of equal states are equal byte for byte
  if (e == hipSuccess) e = hipMemsetAsync(c->base, 0, c->lay.off_small, c->stream);
  if (e == hipSuccess && phi) {
    // porosity plane in the arithmetic type, row pitch applied
    const size_t rs = real_size(c->prec);
    std::vector<char> rows((size_t)c->lay.pitch * p->ny * rs, 0);
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        const double q = phi[(size_t)y * p->nx + x];
        char *dst = rows.data() + ((size_t)y * c->lay.pitch + x) * rs;
        if (rs == 8) std::memcpy(dst, &q, 8);
        else { float f = (float)q; std::memcpy(dst, &f, 4); }
      }
    e = hipMemcpyAsync(c->phi(), rows.data(), rows.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (e == hipSuccess) e = (hipError_t)launch_init(c->prec, c->desc(), stage, stage + n, stage + 2 * n, stage + 3 * n, c->stream);
  // the four device copies of the descriptor the step kernels read
  std::vector<char> dslots(4 * kDescSlot, 0);
  for (int pc = 0; pc < 2; ++pc)
    for (int fc = 0; fc < 2; ++fc) {
      set_parity(c, pc, fc);
      std::memcpy(dslots.data() + (2 * pc + fc) * kDescSlot, c->desc(),
                  c->prec == PREC_FP64 ? sizeof(Desc<double>) : sizeof(Desc<float>));
    }
  set_parity(c, 0, 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->base + c->lay.off_desc, dslots.data(), dslots.size(), hipMemcpyHostToDevice, c->stream);
  // the residual snapshot starts at level 0
  if (e == hipSuccess) e = hipMemcpyAsync(c->snap(), c->d4(), 4 * plane_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->wall_dev(), c->wallT, 4 * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->wall_dev() + 4, c->wallC, 4 * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(stage);
  if (e != hipSuccess) return hip_fail(c, e, "lbm_set_fields");
  c->step = 0;
  c->snap_step = 0;
  c->ready = true;
  c->unstable = false;
  return LBM_OK;
}

// Time steps per launch: default_spl (three for FP32 and FP64 storage, two for FP16), or the
// count set by lbm_set_steps_per_launch, lowered to what the cavity allows.
// With walls through the nodes the two-step kernel places its last tiles against the far
// walls, so the lattice must hold one tile.  FP16 storage with walls through the nodes always
// takes one step per launch: the two-step kernel is slower there (2048^2: 41 against 50
// GLUPS), and its FP16 results would not match the one-step kernel's bit for bit (the
// compiler fuses multiply-adds of the boundary rule differently in the two kernels, and
// stochastic rounding turns a last-bit FP32 difference into a different FP16 value now and
// then).
static bool two_step_ok(const lbm_ctx *c) {
  if (!node_walls(&c->p)) return true;
  if (c->prec == PREC_FP16S) return false;
  int w = 0, h = 0;
  two_step_tile_shape(c->prec, &w, &h);
  return c->p.nx >= w && c->p.ny >= h;
}

// The three-step kernel: FP32 and FP64 storage, walls half a spacing outside.
static bool three_step_ok(const lbm_ctx *c) { return !node_walls(&c->p) && c->prec != PREC_FP16S; }

static int ctx_spl(const lbm_ctx *c) {
  if (!two_step_ok(c)) return 1;
  const int n = c->steps_per_launch > 0 ? c->steps_per_launch : default_spl(c->prec, (double)c->p.nx * c->p.ny);
  return (n == 3 && !three_step_ok(c)) ? 2 : n;
}

static int ctx_policy(const lbm_ctx *c) {
  return c->cache_policy >= 0 ? c->cache_policy : default_policy(c->prec, (double)c->p.nx * c->p.ny, ctx_spl(c));
}

static int ctx_rows(const lbm_ctx *c) {
  if (node_walls(&c->p)) return 8;
  return c->tile_rows > 0 ? c->tile_rows : default_rows(c->prec, (double)c->p.nx * c->p.ny);
}

// the rows each multi-step launch takes: the tile rows apply to FP32's three-step and FP16's
// two-step launch, the others have 8-row tiles
static int rows2_of(const lbm_ctx *c) { return c->prec == PREC_FP16S ? ctx_rows(c) : 8; }
static int rows3_of(const lbm_ctx *c) { return c->prec == PREC_FP32 ? ctx_rows(c) : 8; }

static int ctx_strip(const lbm_ctx *c) {
  if (c->strip >= 0) return c->strip;
  const int spl = ctx_spl(c);
  return default_strip(c->prec, c->p.nx, c->p.ny, spl, spl == 3 ? rows3_of(c) : rows2_of(c));
}

// n steps with plain launches: three or two steps per launch as ctx_spl allows, the remainder
// in shorter launches
static lbm_status step_plain(lbm_ctx *c, int64_t n) {
  const int cp = ctx_policy(c);
  const int spl = ctx_spl(c);
  const int sw = ctx_strip(c), rows2 = rows2_of(c), rows3 = rows3_of(c);
  while (n > 0) {
    set_parity(c, c->cur);
    if (spl == 3 && n >= 3) {
      int e = launch_step3(c->prec, c->desc(), c->desc_dev(c->cur, c->d4cur), cp, 0, sw, rows3, c->stream);
      if (e) return hip_fail(c, (hipError_t)e, "three-step kernel launch");
      c->d4cur ^= 1;
      n -= 3;
    } else if (spl >= 2 && n >= 2) {
      int e = launch_step2(c->prec, c->desc(), c->desc_dev(c->cur, c->d4cur), cp, 0, sw, rows2, c->stream);
      if (e) return hip_fail(c, (hipError_t)e, "two-step kernel launch");
      c->d4cur ^= 1;
      n -= 2;
    } else {
      int e = launch_step(c->prec, c->desc(), c->desc_dev(c->cur, c->d4cur), c->tile, cp, 0, c->stream);
      if (e) return hip_fail(c, (hipError_t)e, "step kernel launch");
      n -= 1;
    }
    c->cur ^= 1;
  }
  return LBM_OK;
}

// Steps per launch and steps per replay of the step graph.  A multi-step launch flips the
// population and the field buffer, a one-step launch the population buffer only; a replay
// must flip each an even number of times, so that it ends on the buffers it started from:
// three steps per launch replay the largest multiple of 6 steps in graph_chunk, two steps per
// launch the whole chunk when it is a multiple of 4; otherwise one step per launch.
static void graph_plan(const lbm_ctx *c, int *spl, int *steps) {
  const int n = ctx_spl(c);
  if (n == 3 && c->graph_chunk >= 6) {
    *spl = 3;
    *steps = c->graph_chunk / 6 * 6;
  } else if (n >= 2 && c->graph_chunk % 4 == 0) {
    *spl = 2;
    *steps = c->graph_chunk;
  } else {
    *spl = 1;
    *steps = c->graph_chunk;
  }
}

// Graph of one replay (graph_plan): its launches in a fixed order.
static lbm_status ensure_graph(lbm_ctx *c) {
  const int cp = ctx_policy(c);
  const int sw = ctx_strip(c), rows = ctx_rows(c), rows2 = rows2_of(c), rows3 = rows3_of(c);
  int spl = 1, gsteps = 0;
  graph_plan(c, &spl, &gsteps);
  if (c->graph && c->graph_cur == c->cur && c->graph_tile.tx == c->tile.tx && c->graph_tile.ty == c->tile.ty &&
      c->graph_cp == cp && c->graph_d4 == c->d4cur && c->graph_spl == spl && c->graph_sw == sw &&
      c->graph_rows == rows)
    return LBM_OK;
  drop_graph(c);
  hipStream_t cs;
  HIP_CHECK(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  const int start = c->cur;
  if (e == hipSuccess) {
    int cur = start, d4 = c->d4cur;
    for (int k = 0; k < gsteps / spl && e == hipSuccess; ++k) {
      set_parity(c, cur, d4);
      if (spl == 3) {
        e = (hipError_t)launch_step3(c->prec, c->desc(), c->desc_dev(cur, d4), cp, 0, sw, rows3, cs);
        d4 ^= 1;
      } else if (spl == 2) {
        e = (hipError_t)launch_step2(c->prec, c->desc(), c->desc_dev(cur, d4), cp, 0, sw, rows2, cs);
        d4 ^= 1;
      } else {
        e = (hipError_t)launch_step(c->prec, c->desc(), c->desc_dev(cur, d4), c->tile, cp, 0, cs);
      }
      cur ^= 1;
    }
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
  }
  set_parity(c, start);
  if (e == hipSuccess) e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    c->graph = nullptr;
    return hip_fail(c, e, "step graph capture");
  }
  c->graph_cur = start;
  c->graph_tile = c->tile;
  c->graph_cp = cp;
  c->graph_d4 = c->d4cur;
  c->graph_spl = spl;
  c->graph_sw = sw;
  c->graph_rows = rows;
  return LBM_OK;
}

LBM_API lbm_status lbm_step(lbm_ctx *c, int64_t nsteps) {
  Range range_("lbm_step");
  if (!c || nsteps < 0) return LBM_EINVAL;
  if (!c->ready) return fail(c, LBM_ESTATE, "lbm_step before lbm_set_fields");
  if (c->batch) return fail(c, LBM_ESTATE, "context is attached to a batch");
  if (c->unstable)
    return fail(c, LBM_ESTATE, "the fields hold a non-finite value (reported at step %lld); restart with "
                "lbm_set_fields or restore a state with lbm_set_state", (long long)c->step);
  int64_t left = nsteps;
  int gspl = 1, gsteps = 0;
  graph_plan(c, &gspl, &gsteps);
  if (c->graph_chunk > 0 && left >= gsteps) {
    lbm_status s = ensure_graph(c);
    if (s != LBM_OK) return s;
    while (left >= gsteps) {
      HIP_CHECK(c, hipGraphLaunch(c->graph, c->stream), "hipGraphLaunch");
      left -= gsteps;   // a replay leaves the current buffers unchanged
    }
  }
  lbm_status s = step_plain(c, left);
  if (s != LBM_OK) return s;
  c->step += nsteps;
  return LBM_OK;
}

// FP64 fields of the current level into host memory through a device staging buffer: `stage`
// (5 nx ny doubles), or one allocated for the call when stage is NULL
static lbm_status export_fields(lbm_ctx *c, double *fields, double *stage = nullptr) {
  set_parity(c, c->cur);
  const size_t n = (size_t)c->p.nx * c->p.ny;
  const bool own = stage == nullptr;
  if (own) HIP_CHECK(c, hipMalloc((void **)&stage, 5 * n * sizeof(double)), "hipMalloc export");
  hipError_t he = (hipError_t)launch_export(c->prec, c->desc(), 0, stage, c->stream);
  if (he == hipSuccess) he = hipMemcpyAsync(fields, stage, 5 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
  if (own) (void)hipFree(stage);
  if (he != hipSuccess) return hip_fail(c, he, "field export");
  return LBM_OK;
}

LBM_API lbm_status lbm_get_fields(lbm_ctx *c, double *fields) {
  if (!c || !fields) return LBM_EINVAL;
  if (!c->ready) return fail(c, LBM_ESTATE, "lbm_get_fields before lbm_set_fields");
  return export_fields(c, fields);
}

// The observables of the current level, with the per-block partial sums in `partials`, the 20
// result slots in `slots` and, when fields is not NULL, the field export staged in `stage`
// (NULL: allocated for the call).
static lbm_status observe(lbm_ctx *c, lbm_obs *out, double *fields, double *partials, double *slots,
                          double *stage) {
  set_parity(c, c->cur);
  const int nb = c->lay.nblocks_obs;
  int e = launch_observables(c->prec, c->desc(), 0, c->snap(), partials, nb, slots, c->wall_dev(),
                             c->wall_dev() + 4, c->dv.dT != 0 ? c->dv.L / c->dv.dT : 0.0,
                             c->dv.dC != 0 ? c->dv.L / c->dv.dC : 0.0, c->stream);
  if (e) return hip_fail(c, (hipError_t)e, "observables launch");
  double r[20];
  HIP_CHECK(c, hipMemcpyAsync(r, slots, sizeof r, hipMemcpyDeviceToHost, c->stream), "observables copy");
  if (fields) {
    lbm_status fs = export_fields(c, fields, stage);
    if (fs != LBM_OK) return fs;
  }
  HIP_CHECK(c, hipStreamSynchronize(c->stream), "observables sync");
  std::memset(out, 0, sizeof *out);
  out->step = c->step;
  out->mass = r[0];
  out->heat = r[1];
  out->solute = r[2];
  const double dn = (double)(c->step - c->snap_step);
  if (dn > 0) {
    out->r_u = std::sqrt(r[3]) / (dn * std::max(std::sqrt(r[4]), 1e-30));
    out->r_T = std::sqrt(r[5]) / (dn * std::max(std::sqrt(r[6]), 1e-30));
    out->r_C = std::sqrt(r[7]) / (dn * std::max(std::sqrt(r[8]), 1e-30));
  }
  out->max_ux = r[9];
  out->max_uy = r[10];
  out->nonfinite = r[11] > 0 || !std::isfinite(r[0]) || !std::isfinite(r[3]);
  for (int s = 0; s < 4; ++s) {
    out->Nu[s] = r[12 + s];
    out->Sh[s] = r[16 + s];
  }
  c->snap_step = c->step;
  if (out->nonfinite) {
    c->unstable = true;
    return fail(c, LBM_EUNSTABLE, "non-finite value in the fields at step %lld", (long long)c->step);
  }
  return LBM_OK;
}

LBM_API lbm_status lbm_observables(lbm_ctx *c, lbm_obs *out, double *fields) {
  Range range_("lbm_observables");
  if (!c || !out) return LBM_EINVAL;
  if (!c->ready) return fail(c, LBM_ESTATE, "lbm_observables before lbm_set_fields");
  return observe(c, out, fields, c->partials(), c->obs_out(), nullptr);
}

LBM_API lbm_status lbm_observables_static(lbm_ctx *c, lbm_obs *out, double *fields) {
  Range range_("lbm_observables_static");
  if (!c || !out) return LBM_EINVAL;
  if (!c->ready) return fail(c, LBM_ESTATE, "lbm_observables_static before lbm_set_fields");
  if (!c->scratch) return fail(c, LBM_EDEVICE, "no fixed scratch on this device");
  const StaticScratchLayout L = static_scratch_layout();
  if (c->p.ny > L.max_rows)
    return fail(c, LBM_EINVAL, "lbm_observables_static serves lattices of at most %d rows (this one has %d)",
                L.max_rows, c->p.ny);
  if (fields && (long long)c->p.nx * c->p.ny > L.max_nodes)
    return fail(c, LBM_EINVAL, "lbm_observables_static exports the fields of lattices of at most %lld nodes "
                "(this one has %lld)", L.max_nodes, (long long)c->p.nx * c->p.ny);
  return observe(c, out, fields, c->scratch + L.partials, c->scratch + L.out, c->scratch + L.fields);
}

LBM_API lbm_status lbm_get_derived(const lbm_ctx *c, lbm_derived *out) {
  if (!c || !out) return LBM_EINVAL;
  if (!c->ready) return LBM_ESTATE;
  *out = c->dv;
  return LBM_OK;
}

// ---- checkpoints ---------------------------------------------------------------------
namespace {
struct StateHeader {
  char magic[8];
  int32_t nx, ny, precision;
  uint32_t counter;          // device step counter of the stored state
  int64_t step, snap_step;
  uint64_t pop_bytes, d4_bytes;
};
}  // namespace

LBM_API uint64_t lbm_state_bytes(const lbm_ctx *c) {
  if (!c) return 0;
  const size_t es = store_size(c->prec), rs = real_size(c->prec);
  return sizeof(StateHeader) + (uint64_t)NPOP * c->lay.plane * es + 2ull * ND4 * c->lay.plane * rs;
}

LBM_API lbm_status lbm_get_state(lbm_ctx *c, void *host, uint64_t bytes) {
  if (!c || !host) return LBM_EINVAL;
  if (!c->ready) return fail(c, LBM_ESTATE, "no state before lbm_set_fields");
  if (bytes < lbm_state_bytes(c)) return fail(c, LBM_EINVAL, "buffer too small");
  StateHeader h{};
  std::memcpy(h.magic, "LBMDDPS3", 8);
  h.nx = c->p.nx;
  h.ny = c->p.ny;
  h.precision = c->prec;
  h.step = c->step;
  h.snap_step = c->snap_step;
  h.pop_bytes = (uint64_t)NPOP * c->lay.plane * store_size(c->prec);
  h.d4_bytes = (uint64_t)ND4 * c->lay.plane * real_size(c->prec);
  HIP_CHECK(c, hipMemcpyAsync(&h.counter, c->counter() + c->cur, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream),
            "state copy");
  HIP_CHECK(c, hipStreamSynchronize(c->stream), "state sync");
  char *dst = (char *)host;
  std::memcpy(dst, &h, sizeof h);
  dst += sizeof h;
  HIP_CHECK(c, hipMemcpyAsync(dst, c->pop(c->cur), h.pop_bytes, hipMemcpyDeviceToHost, c->stream), "state copy");
  HIP_CHECK(c, hipMemcpyAsync(dst + h.pop_bytes, c->d4(), h.d4_bytes, hipMemcpyDeviceToHost, c->stream), "state copy");
  HIP_CHECK(c, hipMemcpyAsync(dst + h.pop_bytes + h.d4_bytes, c->snap(), h.d4_bytes, hipMemcpyDeviceToHost, c->stream),
            "state copy");
  HIP_CHECK(c, hipStreamSynchronize(c->stream), "state sync");
  return LBM_OK;
}

LBM_API lbm_status lbm_set_state(lbm_ctx *c, const void *host, uint64_t bytes) {
  if (!c || !host) return LBM_EINVAL;
  if (!c->ready) return fail(c, LBM_ESTATE, "lbm_set_fields must run first (it fixes the porosity)");
  if (c->batch) return fail(c, LBM_ESTATE, "context is attached to a batch");
  if (bytes < lbm_state_bytes(c)) return fail(c, LBM_EINVAL, "buffer too small");
  StateHeader h;
  std::memcpy(&h, host, sizeof h);
  if (std::memcmp(h.magic, "LBMDDPS3", 8) != 0 || h.nx != c->p.nx || h.ny != c->p.ny || h.precision != c->prec ||
      h.pop_bytes != (uint64_t)NPOP * c->lay.plane * store_size(c->prec) ||
      h.d4_bytes != (uint64_t)ND4 * c->lay.plane * real_size(c->prec))
    return fail(c, LBM_EINVAL, "state does not match this context");
  const char *src = (const char *)host + sizeof h;
  drop_graph(c);
  c->cur = 0;
  c->d4cur = 0;
  set_parity(c, 0);
  HIP_CHECK(c, hipMemcpyAsync(c->pop(0), src, h.pop_bytes, hipMemcpyHostToDevice, c->stream), "state copy");
  HIP_CHECK(c, hipMemcpyAsync(c->counter(), &h.counter, sizeof(unsigned), hipMemcpyHostToDevice, c->stream),
            "state copy");
  HIP_CHECK(c, hipMemcpyAsync(c->d4(), src + h.pop_bytes, h.d4_bytes, hipMemcpyHostToDevice, c->stream), "state copy");
  HIP_CHECK(c, hipMemcpyAsync(c->snap(), src + h.pop_bytes + h.d4_bytes, h.d4_bytes, hipMemcpyHostToDevice, c->stream),
            "state copy");
  HIP_CHECK(c, hipStreamSynchronize(c->stream), "state sync");
  c->step = h.step;
  c->snap_step = h.snap_step;
  c->unstable = false;
  return LBM_OK;
}

// ---- launch shape and autotuning ---------------------------------------------------------
static bool tile_supported(int tx, int ty) {
  return (tx == 64 || tx == 128 || tx == 256) && (ty == 1 || ty == 2 || ty == 4 || ty == 8);
}

LBM_API lbm_status lbm_set_tile(lbm_ctx *c, int32_t tx, int32_t ty) {
  if (!c) return LBM_EINVAL;
  if (tx == 0 && ty == 0) {
    c->tile = default_tile(&c->p);
    return LBM_OK;
  }
  if (!tile_supported(tx, ty)) return fail(c, LBM_EINVAL, "unsupported tile %dx%d", tx, ty);
  c->tile = Tile{tx, ty};
  return LBM_OK;
}

LBM_API lbm_status lbm_set_graph_chunk(lbm_ctx *c, int32_t chunk) {
  if (!c) return LBM_EINVAL;
  if (chunk < 0 || chunk == 1 || (chunk & 1)) return fail(c, LBM_EINVAL, "graph chunk must be 0 or even >= 2");
  if (chunk != c->graph_chunk) drop_graph(c);
  c->graph_chunk = chunk;
  return LBM_OK;
}

LBM_API lbm_status lbm_get_tile(const lbm_ctx *c, int32_t *tx, int32_t *ty) {
  if (!c || !tx || !ty) return LBM_EINVAL;
  *tx = c->tile.tx;
  *ty = c->tile.ty;
  return LBM_OK;
}

LBM_API lbm_status lbm_set_cache_policy(lbm_ctx *c, int32_t policy) {
  if (!c) return LBM_EINVAL;
  if (policy < -1 || policy >= CP_COUNT) return fail(c, LBM_EINVAL, "unknown cache policy %d", policy);
  c->cache_policy = policy;
  return LBM_OK;
}

LBM_API int32_t lbm_get_cache_policy(const lbm_ctx *c) { return c ? ctx_policy(c) : -1; }

LBM_API lbm_status lbm_set_strip_width(lbm_ctx *c, int32_t tiles) {
  if (!c) return LBM_EINVAL;
  if (tiles < -1 || tiles > 1024) return fail(c, LBM_EINVAL, "strip width must be -1 (default), 0 or 1..1024 tiles");
  c->strip = tiles;
  return LBM_OK;
}

LBM_API int32_t lbm_get_strip_width(const lbm_ctx *c) { return c ? ctx_strip(c) : -1; }

LBM_API lbm_status lbm_set_tile_rows(lbm_ctx *c, int32_t rows) {
  if (!c) return LBM_EINVAL;
  if (rows != 0 && rows != 8 && !(rows == 12 && c->prec != PREC_FP64))
    return fail(c, LBM_EINVAL, "tile rows must be 0 (default), 8 or, with FP32 and FP16 storage, 12");
  c->tile_rows = rows;
  return LBM_OK;
}

// the rows of the multi-step launch in effect (8 where the steps per launch leave no tile rows to
// choose)
LBM_API int32_t lbm_get_tile_rows(const lbm_ctx *c) {
  if (!c) return 0;
  const int spl = ctx_spl(c);
  return spl == 3 ? rows3_of(c) : spl == 2 ? rows2_of(c) : 8;
}

LBM_API lbm_status lbm_set_steps_per_launch(lbm_ctx *c, int32_t n) {
  if (!c) return LBM_EINVAL;
  if (n < 0 || n > 3) return fail(c, LBM_EINVAL, "steps per launch must be 0 (default), 1, 2 or 3");
  c->steps_per_launch = n;
  return LBM_OK;
}

LBM_API int32_t lbm_get_steps_per_launch(const lbm_ctx *c) { return c ? ctx_spl(c) : 0; }

LBM_API lbm_status lbm_autotune(lbm_ctx *c, int32_t steps, int32_t *tx_out, int32_t *ty_out, double *ms_out) {
  Range range_("lbm_autotune");
  if (!c || steps < 2) return LBM_EINVAL;
  if (!c->ready) return fail(c, LBM_ESTATE, "lbm_autotune before lbm_set_fields");
  if (c->batch) return fail(c, LBM_ESTATE, "context is attached to a batch");
  // save the state on the device, try each shape, restore
  const size_t pop_bytes = (size_t)NPOP * c->lay.plane * store_size(c->prec);
  const size_t d4_bytes = (size_t)ND4 * c->lay.plane * real_size(c->prec);
  char *save = nullptr;
  HIP_CHECK(c, hipMalloc((void **)&save, pop_bytes + d4_bytes + 2 * sizeof(unsigned)), "hipMalloc autotune");
  const int cur0 = c->cur;
  const int64_t step0 = c->step;
  const Tile tile0 = c->tile;
  const int cp0 = c->cache_policy, spl0 = c->steps_per_launch, d4cur0 = c->d4cur, sw0 = c->strip;
  const int rows0 = c->tile_rows;
  hipError_t e = hipMemcpyAsync(save, c->pop(cur0), pop_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(save + pop_bytes, c->d4(), d4_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(save + pop_bytes + d4_bytes, c->counter(), 2 * sizeof(unsigned), hipMemcpyDeviceToDevice, c->stream);
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  double best = 1e300;
  Tile best_tile = tile0;
  int best_cp = ctx_policy(c), best_spl = ctx_spl(c), best_sw = c->strip, best_rows = c->tile_rows;
  const int txs[] = {64, 128, 256};
  const int tys[] = {1, 2, 4, 8};
  struct Cand {
    int spl, cp, tx, ty, sw, rows;
  };
  std::vector<Cand> cands;
  for (int cp = 0; cp < CP_COUNT; ++cp)
    for (int tx : txs)
      for (int ty : tys) cands.push_back(Cand{1, cp, tx, ty, sw0, rows0});
  // the multi-step kernels have a fixed tile (64 x 8, FP64 32 x 8); their tile order: row by row
  // or strips of 4 or 8 tiles, where the lattice is wider than the strip
  int w2 = 0, h2 = 0;
  two_step_tile_shape(c->prec, &w2, &h2);
  const int ntx2 = (c->p.nx + w2 - 1) / w2;
  std::vector<int> sws{0};
  for (int sw : {4, 8})
    if (ntx2 > sw) sws.push_back(sw);
  const int aligned = ntx2 % 8 == 0 ? ntx2 / 8 : 0;   // one strip per XCD band
  if (aligned >= 3 && aligned <= 16 && aligned != 4 && aligned != 8) sws.push_back(aligned);
  if (two_step_ok(c))
    for (int rows : {8, 12}) {   // FP16 without node walls: the 64 x 8 and the 64 x 12 tile
      if (rows == 12 && (c->prec != PREC_FP16S || node_walls(&c->p))) continue;
      for (int cp = 0; cp < CP_COUNT; ++cp)
        for (int sw : sws) cands.push_back(Cand{2, cp, tile0.tx, tile0.ty, sw, rows});
    }
  if (three_step_ok(c))   // FP32: the 64 x 8 and the 64 x 12 tile
    for (int rows : {8, 12}) {
      if (rows == 12 && c->prec != PREC_FP32) continue;
      for (int cp = 0; cp < CP_COUNT; ++cp)
        for (int sw : sws) cands.push_back(Cand{3, cp, tile0.tx, tile0.ty, sw, rows});
    }
  const int nsteps = (steps + 5) / 6 * 6;   // whole launches of two and of three steps
  for (const Cand &k : cands) {
    if (e != hipSuccess) break;
    c->tile = Tile{k.tx, k.ty};
    c->cache_policy = k.cp;
    c->steps_per_launch = k.spl;
    c->strip = k.sw;
    c->tile_rows = k.rows;
    if (step_plain(c, 6) != LBM_OK) { e = hipErrorUnknown; break; }   // warm-up
    e = hipEventRecord(t0, c->stream);
    if (e == hipSuccess && step_plain(c, nsteps) != LBM_OK) e = hipErrorUnknown;
    if (e == hipSuccess) e = hipEventRecord(t1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess && ms / nsteps < best) {
      best = ms / nsteps;
      best_tile = c->tile;
      best_cp = k.cp;
      best_spl = k.spl;
      best_sw = k.sw;
      best_rows = k.rows;
    }
  }
  // restore
  c->cur = cur0;
  c->d4cur = d4cur0;
  set_parity(c, cur0);
  if (e == hipSuccess) e = hipMemcpyAsync(c->pop(cur0), save, pop_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d4(), save + pop_bytes, d4_bytes, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->counter(), save + pop_bytes + d4_bytes, 2 * sizeof(unsigned), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(save);
  c->step = step0;
  if (e != hipSuccess) {
    c->tile = tile0;
    c->cache_policy = cp0;
    c->steps_per_launch = spl0;
    c->strip = sw0;
    c->tile_rows = rows0;
    return hip_fail(c, e, "autotune");
  }
  c->tile = best_tile;
  c->cache_policy = best_cp;
  c->steps_per_launch = best_spl;
  c->strip = best_sw;
  c->tile_rows = best_rows;
  drop_graph(c);
  if (tx_out) *tx_out = best_tile.tx;
  if (ty_out) *ty_out = best_tile.ty;
  if (ms_out) *ms_out = best;
  return LBM_OK;
}

// ================================================================== batch
// A group: cavities of one precision whose step touches at most kGroupBytes together, so
// that they stay in the Infinity Cache while the group advances a chunk of steps; items
// [first, first + count) of the precision's item table.
struct BatchGroup {
  int prec, cls, cp, first, count, first2, count2;   // one-step items, multi-step items
  int grid2;   // work-groups of the multi-step launch (one per item; count2 rounded up to a
               // power of two, so that a graph survives small changes of the group)
  int shape;   // tile shape of the multi-step items (batch_tile_shape)
  int spl;     // steps per multi-step launch: 3, 2, or 1 (one-step launches only)
  int nee;     // walls through the boundary nodes: two-step launches only, last tiles against
               // the far walls; a remaining single step runs as the cavity's own launch
};

// Launch choice of the groups of one precision and size class: the two-step tile shape, or
// kBatchThree for three steps per launch on the three-step tile (shape 0), and the cache
// policy (-1: the default rule); set by lbm_batch_set_tile or lbm_batch_autotune.
struct BatchChoice {
  int shape = 0, cp = -1;
};
int batch_three_shape() { return batch_tile_shapes(); }

// size classes of cavities in a batch, by width: <= 64, <= 128, <= 256, wider
constexpr int kBatchClasses = 4;
int batch_class(int nx) { return nx <= 64 ? 0 : nx <= 128 ? 1 : nx <= 256 ? 2 : 3; }

struct lbm_batch {
  int cap = 0;
  int chunk = 2;
  hipStream_t stream = nullptr;
  std::vector<lbm_ctx *> ctx;
  // per precision: descriptor table and item tables (device): one-step tiles and the tiles of
  // the multi-step launches
  void *descs[3] = {nullptr, nullptr, nullptr};
  Item *items[3] = {nullptr, nullptr, nullptr};
  Item *items2[3] = {nullptr, nullptr, nullptr};
  int item_cap[3] = {0, 0, 0};
  int item2_cap[3] = {0, 0, 0};
  std::vector<BatchGroup> groups;
  BatchChoice choice[3][kBatchClasses];   // per precision and size class
  int *ranges = nullptr;     // device: {first, count, first2, count2} per group
  int range_cap = 0;
  int grid = 2048;           // work-groups of the one-step batched launch
  hipGraphExec_t graph = nullptr;
  std::vector<int> graph_key;   // (precision, cache policy) of each group when the graph was captured
  bool dirty = true;
};

namespace {

constexpr double kGroupBytes = 200e6;   // per-step bytes of one group (Infinity Cache: 256 MB)

// Steps per batched two-step launch: 2 when a replay chunk is a multiple of 4 steps (so a
// replay flips the population and field buffers an even number of times), else 1.
int batch_spl(const lbm_batch *b) { return b->chunk % 4 == 0 ? 2 : 1; }

// three steps per launch need a chunk that is a multiple of 6 (an even number of launches)
// and of 4 (the two-step groups of the same replay): of 12; FP32 and FP64 storage only
bool batch_three_ok(const lbm_batch *b, int prec) { return b->chunk % 12 == 0 && prec != PREC_FP16S; }

// steps per multi-step launch of the groups of one precision under a launch choice
int batch_group_spl(const lbm_batch *b, int prec, const BatchChoice &ch) {
  if (ch.shape == batch_three_shape() && batch_three_ok(b, prec)) return 3;
  return batch_spl(b);
}

// steps per multi-step launch of an attached cavity (its group's)
int batch_ctx_spl(const lbm_batch *b, const lbm_ctx *c) {
  if (node_walls(&c->p)) return 2;
  return batch_group_spl(b, c->prec, b->choice[c->prec][batch_class(c->p.nx)]);
}

void drop_batch_graph(lbm_batch *b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_key.clear();
}

lbm_status batch_upload(lbm_batch *b) {
  b->groups.clear();
  for (int prec = 0; prec < 3; ++prec) {
    std::vector<Item> items, items2;
    std::vector<Desc<double>> d64;
    std::vector<Desc<float>> d32;
    double gnodes = 0;
    // cavities of this precision by size class, those with walls through the nodes after the
    // others of their class (attach order within each)
    std::vector<lbm_ctx *> order;
    for (int cls = 0; cls < kBatchClasses; ++cls)
      for (int nee = 0; nee < 2; ++nee)
        for (lbm_ctx *c : b->ctx)
          if (c->prec == prec && batch_class(c->p.nx) == cls && (int)node_walls(&c->p) == nee) order.push_back(c);
    for (lbm_ctx *c : order) {
      const int cls = batch_class(c->p.nx);
      const int nee = node_walls(&c->p) ? 1 : 0;
      const BatchChoice &ch = b->choice[prec][cls];
      const int idx = prec == PREC_FP64 ? (int)d64.size() : (int)d32.size();
      set_parity(c, c->cur);
      if (prec == PREC_FP64) d64.push_back(c->d64);
      else d32.push_back(c->d32);
      // groups per size class, closed when the next cavity would take the group past
      // kGroupBytes (a larger cavity is a group of its own)
      const double nodes = (double)c->p.nx * c->p.ny;
      if (b->groups.empty() || b->groups.back().prec != prec || b->groups.back().cls != cls ||
          b->groups.back().nee != nee || (gnodes > 0 && (gnodes + nodes) * bytes_per_lu(prec) > kGroupBytes)) {
        // node-wall groups: two steps per launch on the two-step tile (attach checked that the
        // chunk allows two steps and that the cavity holds one tile)
        const int spl = nee ? 2 : batch_group_spl(b, prec, ch);
        b->groups.push_back(BatchGroup{prec, cls, 0, (int)items.size(), 0, (int)items2.size(), 0, 1,
                                       (spl == 3 || nee) ? 0 : ch.shape, spl, nee});
        gnodes = 0;
      }
      gnodes += nodes;
      int w2 = 0, h2 = 0;
      batch_tile_shape(prec, b->groups.back().shape, &w2, &h2);
      // 256-thread tiles of tw x (256/tw) nodes; tw in {256, 128, 64} wastes the fewest
      // lanes on the ragged right edge (ties go to the wider tile)
      int tw = 256;
      for (int cand : {128, 64})
        if ((c->p.nx + cand - 1) / cand * cand < (c->p.nx + tw - 1) / tw * tw) tw = cand;
      const int rows = 256 / tw;
      const int ntx = (c->p.nx + tw - 1) / tw, nty = (c->p.ny + rows - 1) / rows;
      for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) items.push_back(Item{idx, tx * tw, ty * rows, tw});
      const int ntx2 = (c->p.nx + w2 - 1) / w2, nty2 = (c->p.ny + h2 - 1) / h2;
      for (int ty = 0; ty < nty2; ++ty)
        for (int tx = 0; tx < ntx2; ++tx) {
          int x0 = tx * w2, y0 = ty * h2;
          if (nee) {   // as the single-cavity two-step kernel: the last tiles against the far walls
            x0 = std::min(x0, c->p.nx - w2);
            y0 = std::min(y0, c->p.ny - h2);
          }
          items2.push_back(Item{idx, x0, y0, w2});
        }
      BatchGroup &g = b->groups.back();
      g.count = (int)items.size() - g.first;
      g.count2 = (int)items2.size() - g.first2;
      g.grid2 = 1;
      while (g.grid2 < g.count2) g.grid2 *= 2;
      g.cp = ch.cp >= 0 ? ch.cp : default_policy(prec, gnodes, g.spl);
    }
    const int n = (int)items.size();
    if (n > b->item_cap[prec]) {
      // grow the item table; the graph references the old pointer, so drop it
      drop_batch_graph(b);
      if (b->items[prec]) (void)hipFree(b->items[prec]);
      b->items[prec] = nullptr;
      int cap = std::max(n, 2 * b->item_cap[prec]);
      b->item_cap[prec] = 0;
      if (hipMalloc((void **)&b->items[prec], (size_t)cap * sizeof(Item)) != hipSuccess) {
        b->items[prec] = nullptr;
        return LBM_ENOMEM;
      }
      b->item_cap[prec] = cap;
    }
    const int n2 = (int)items2.size();
    if (n2 > b->item2_cap[prec]) {
      drop_batch_graph(b);
      if (b->items2[prec]) (void)hipFree(b->items2[prec]);
      b->items2[prec] = nullptr;
      int cap = std::max(n2, 2 * b->item2_cap[prec]);
      b->item2_cap[prec] = 0;
      if (hipMalloc((void **)&b->items2[prec], (size_t)cap * sizeof(Item)) != hipSuccess) {
        b->items2[prec] = nullptr;
        return LBM_ENOMEM;
      }
      b->item2_cap[prec] = cap;
    }
    if (n2 && hipMemcpyAsync(b->items2[prec], items2.data(), n2 * sizeof(Item), hipMemcpyHostToDevice, b->stream) !=
                  hipSuccess)
      return LBM_EDEVICE;
    if (n) {
      if (hipMemcpyAsync(b->items[prec], items.data(), n * sizeof(Item), hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return LBM_EDEVICE;
      const void *src = prec == PREC_FP64 ? (const void *)d64.data() : (const void *)d32.data();
      const size_t bytes = prec == PREC_FP64 ? d64.size() * sizeof(Desc<double>) : d32.size() * sizeof(Desc<float>);
      if (hipMemcpyAsync(b->descs[prec], src, bytes, hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return LBM_EDEVICE;
    }
    // the host copies read host vectors that die at the end of this iteration: wait for them
    if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EDEVICE;
  }
  const int ng = (int)b->groups.size();
  if (ng > b->range_cap) {
    drop_batch_graph(b);   // the graph references the old ranges
    if (b->ranges) (void)hipFree(b->ranges);
    b->ranges = nullptr;
    const int cap = std::max(ng, 2 * b->range_cap);
    b->range_cap = 0;
    if (hipMalloc((void **)&b->ranges, (size_t)cap * 4 * sizeof(int)) != hipSuccess) {
      b->ranges = nullptr;
      return LBM_ENOMEM;
    }
    b->range_cap = cap;
  }
  std::vector<int> r;
  for (const BatchGroup &g : b->groups) {
    r.push_back(g.first);
    r.push_back(g.count);
    r.push_back(g.first2);
    r.push_back(g.count2);
  }
  if (ng && hipMemcpyAsync(b->ranges, r.data(), r.size() * sizeof(int), hipMemcpyHostToDevice, b->stream) != hipSuccess)
    return LBM_EDEVICE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_EDEVICE;
  b->dirty = false;
  return LBM_OK;
}

// (precision, cache policy, two-step grid) of each group: a captured graph stays valid while
// this is unchanged
std::vector<int> batch_key(const lbm_batch *b) {
  std::vector<int> k;
  for (const BatchGroup &g : b->groups) {
    k.push_back(g.prec);
    k.push_back(g.cp);
    k.push_back(g.grid2);
    k.push_back(g.shape);
    k.push_back(g.spl);
  }
  return k;
}

// n steps of group gi: multi-step launches (g.spl steps each) while n allows, then single
// steps.  A multi-step launch flips the population and the field buffers; a single step
// flips the population buffers and updates the current field buffer in place.
hipError_t batch_launch_group(lbm_batch *b, size_t gi, int64_t n, hipStream_t s) {
  const BatchGroup &g = b->groups[gi];
  const int *rg = b->ranges + 4 * gi;
  int64_t k = 0, multi = 0;
  if (g.spl >= 2)
    for (; k + g.spl <= n; k += g.spl, ++multi) {
      const int q = (int)(multi & 1);
      const int e = g.nee      ? launch_step2_batch_nee(g.prec, g.cp, b->descs[g.prec], b->items2[g.prec], rg + 2,
                                                        g.grid2, q, s)
                    : g.spl == 3 ? launch_step3_batch(g.prec, g.cp, b->descs[g.prec], b->items2[g.prec], rg + 2,
                                                      g.grid2, q, s)
                                 : launch_step2_batch(g.prec, g.cp, g.shape, b->descs[g.prec], b->items2[g.prec],
                                                      rg + 2, g.grid2, q, s);
      if (e) return (hipError_t)e;
    }
  // a remaining single step of a node-wall group is the cavity's own one-step launch (the
  // batched one-step kernel has no perimeter work), taken by lbm_batch_step after this call
  if (g.nee) return hipSuccess;
  for (int64_t single = 0; k < n; ++k, ++single) {
    const int parity = (int)((multi + single) & 1) | (int)((multi & 1) << 1);
    int e = launch_step_batch(g.prec, g.cp, b->descs[g.prec], b->items[g.prec], rg, b->grid, parity, s);
    if (e) return (hipError_t)e;
  }
  return hipSuccess;
}

// n steps of every group, group after group (a group's cavities stay cache resident while it
// advances; groups are independent, so the order changes no result)
hipError_t batch_launch_steps(lbm_batch *b, int64_t n, hipStream_t s) {
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    const hipError_t e = batch_launch_group(b, gi, n, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

LBM_API lbm_status lbm_batch_create(int32_t max_cavities, int32_t chunk, void *stream, lbm_batch **out) {
  if (!out || max_cavities < 1 || chunk < 2 || (chunk & 1)) return LBM_EINVAL;
  lbm_batch *b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ENOMEM;
  b->cap = max_cavities;
  b->chunk = chunk;
  b->stream = (hipStream_t)stream;
  int dev = 0;
  std::string arch;
  if (hipGetDevice(&dev) != hipSuccess || !arch_ok(dev, arch)) {
    delete b;
    return LBM_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    b->grid = prop.multiProcessorCount * 8;
  }
  bool ok = true;
  for (int prec = 0; prec < 3 && ok; ++prec) {
    const size_t dsz = prec == PREC_FP64 ? sizeof(Desc<double>) : sizeof(Desc<float>);
    ok = hipMalloc(&b->descs[prec], dsz * max_cavities) == hipSuccess;
  }
  if (!ok) {
    lbm_batch_destroy(b);
    return LBM_ENOMEM;
  }
  *out = b;
  return LBM_OK;
}

LBM_API void lbm_batch_destroy(lbm_batch *b) {
  if (!b) return;
  // the contexts go back to their own streams: let the work queued on the batch's finish first
  (void)hipStreamSynchronize(b->stream);
  for (lbm_ctx *c : b->ctx) {
    c->batch = nullptr;
    c->stream = (hipStream_t)c->p.stream;
  }
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  for (int prec = 0; prec < 3; ++prec) {
    if (b->descs[prec]) (void)hipFree(b->descs[prec]);
    if (b->items[prec]) (void)hipFree(b->items[prec]);
    if (b->items2[prec]) (void)hipFree(b->items2[prec]);
  }
  if (b->ranges) (void)hipFree(b->ranges);
  delete b;
}

LBM_API lbm_status lbm_batch_attach(lbm_batch *b, lbm_ctx *c) {
  if (!b || !c) return LBM_EINVAL;
  if (!c->ready) return fail(c, LBM_ESTATE, "attach before lbm_set_fields");
  if (c->batch) return fail(c, LBM_ESTATE, "context already in a batch");
  if (c->unstable) return fail(c, LBM_ESTATE, "the fields hold a non-finite value");
  if ((int)b->ctx.size() >= b->cap) return fail(c, LBM_ENOMEM, "batch is full");
  if (node_walls(&c->p)) {
    // node-wall cavities advance two steps per batched launch on the two-step tile, placed
    // against the far walls: FP32 and FP64 storage, at least one tile, a chunk that allows two
    // steps per launch
    int w = 0, h = 0;
    two_step_tile_shape(c->prec, &w, &h);
    if (c->prec == PREC_FP16S)
      return fail(c, LBM_EINVAL, "FP16 storage with walls through the boundary nodes is not batched");
    if (c->p.nx < w || c->p.ny < h)
      return fail(c, LBM_EINVAL, "walls through the boundary nodes on a lattice smaller than one two-step tile "
                                 "(%d x %d) are not batched", w, h);
    if (batch_spl(b) != 2)
      return fail(c, LBM_EINVAL, "walls through the boundary nodes are not batched with a chunk that is not a "
                                 "multiple of 4");
  }
  // make prior work of the context visible to the batch stream
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, LBM_EDEVICE, "sync before attach");
  c->batch = b;
  c->stream = b->stream;
  drop_graph(c);
  b->ctx.push_back(c);
  b->dirty = true;
  return LBM_OK;
}

// drops `c` from the batch's list and gives it back its own stream (the caller has waited for
// the batch's queued work)
static void batch_forget(lbm_batch *b, lbm_ctx *c) {
  auto it = std::find(b->ctx.begin(), b->ctx.end(), c);
  if (it != b->ctx.end()) b->ctx.erase(it);
  c->batch = nullptr;
  c->stream = (hipStream_t)c->p.stream;
  b->dirty = true;
}

LBM_API lbm_status lbm_batch_detach(lbm_batch *b, lbm_ctx *c) {
  if (!b || !c) return LBM_EINVAL;
  auto it = std::find(b->ctx.begin(), b->ctx.end(), c);
  if (it == b->ctx.end()) return fail(c, LBM_EINVAL, "context is not in this batch");
  if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(c, LBM_EDEVICE, "sync before detach");
  batch_forget(b, c);
  return LBM_OK;
}

LBM_API int32_t lbm_batch_size(const lbm_batch *b) { return b ? (int32_t)b->ctx.size() : 0; }

LBM_API lbm_status lbm_batch_set_tile(lbm_batch *b, int32_t precision, int32_t size_class, int32_t shape,
                                      int32_t policy) {
  if (!b || precision < 0 || precision > 2 || size_class < 0 || size_class >= kBatchClasses || shape < 0 ||
      shape > batch_three_shape() || (shape == batch_three_shape() && precision == PREC_FP16S) || policy < -1 ||
      policy >= CP_COUNT)
    return LBM_EINVAL;
  b->choice[precision][size_class] = BatchChoice{shape, policy};
  b->dirty = true;
  return LBM_OK;
}

LBM_API lbm_status lbm_batch_autotune(lbm_batch *b, int32_t steps, int32_t *shape_out, int32_t *policy_out) {
  Range range_("lbm_batch_autotune");
  if (!b || steps < 1) return LBM_EINVAL;
  if (b->ctx.empty()) return LBM_OK;
  // whole numbers of pairs of two- and of three-step launches: buffers end where they began
  const int64_t n = (steps + 11) / 12 * 12;
  // save every attached state (current populations, fields, step counters) on the device
  std::vector<size_t> off;
  size_t total = 0;
  for (lbm_ctx *c : b->ctx) {
    off.push_back(total);
    total += round_up((size_t)NPOP * c->lay.plane * store_size(c->prec), 256) +
             round_up((size_t)ND4 * c->lay.plane * real_size(c->prec), 256) + 256;
  }
  char *save = nullptr;
  if (hipMalloc((void **)&save, total) != hipSuccess) return LBM_ENOMEM;
  auto copy_states = [&](bool restore) -> hipError_t {
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < b->ctx.size() && e == hipSuccess; ++i) {
      lbm_ctx *c = b->ctx[i];
      const size_t pb = (size_t)NPOP * c->lay.plane * store_size(c->prec);
      const size_t fb = (size_t)ND4 * c->lay.plane * real_size(c->prec);
      char *dst = save + off[i];
      char *pop = (char *)c->pop(c->cur), *d4 = (char *)c->d4(), *cnt = (char *)c->counter();
      const hipMemcpyKind k = hipMemcpyDeviceToDevice;
      e = restore ? hipMemcpyAsync(pop, dst, pb, k, b->stream) : hipMemcpyAsync(dst, pop, pb, k, b->stream);
      dst += round_up(pb, 256);
      if (e == hipSuccess)
        e = restore ? hipMemcpyAsync(d4, dst, fb, k, b->stream) : hipMemcpyAsync(dst, d4, fb, k, b->stream);
      dst += round_up(fb, 256);
      if (e == hipSuccess)
        e = restore ? hipMemcpyAsync(cnt, dst, 2 * sizeof(unsigned), k, b->stream)
                    : hipMemcpyAsync(dst, cnt, 2 * sizeof(unsigned), k, b->stream);
    }
    return e;
  };
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = copy_states(false);
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  lbm_status st = LBM_OK;
  // one step per launch: no multi-step tile; three steps per launch where the chunk allows
  const int two_shapes = batch_spl(b) == 2 ? batch_tile_shapes() : 1;
  for (int prec = 0; prec < 3 && e == hipSuccess && st == LBM_OK; ++prec)
    for (int cls = 0; cls < kBatchClasses && e == hipSuccess && st == LBM_OK; ++cls) {
      bool present = false;
      for (lbm_ctx *c : b->ctx) present |= c->prec == prec && batch_class(c->p.nx) == cls;
      if (!present) continue;
      float best = 3e38f;
      BatchChoice keep = b->choice[prec][cls];
      const int shapes = two_shapes + (batch_three_ok(b, prec) ? 1 : 0);
      for (int k = 0; k < shapes && e == hipSuccess && st == LBM_OK; ++k)
        for (int cp = 0; cp < CP_COUNT && e == hipSuccess && st == LBM_OK; ++cp) {
          const int shape = k < two_shapes ? k : batch_three_shape();
          b->choice[prec][cls] = BatchChoice{shape, cp};
          st = batch_upload(b);
          if (st != LBM_OK) break;
          // warm-up, then the timed steps, of this class's groups only
          for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
            if (pass == 1) e = hipEventRecord(t0, b->stream);
            for (size_t gi = 0; gi < b->groups.size() && e == hipSuccess; ++gi)
              if (b->groups[gi].prec == prec && b->groups[gi].cls == cls)
                e = batch_launch_group(b, gi, pass == 0 ? 12 : n, b->stream);
          }
          if (e == hipSuccess) e = hipEventRecord(t1, b->stream);
          if (e == hipSuccess) e = hipEventSynchronize(t1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
          if (e == hipSuccess) e = copy_states(true);
          if (e == hipSuccess && ms < best) {
            best = ms;
            keep = b->choice[prec][cls];
          }
        }
      b->choice[prec][cls] = keep;
      if (shape_out) shape_out[prec * kBatchClasses + cls] = keep.shape;
      if (policy_out) policy_out[prec * kBatchClasses + cls] = keep.cp;
    }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(save);
  drop_batch_graph(b);
  b->dirty = true;
  if (st != LBM_OK) return st;
  return e == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

LBM_API lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps) {
  Range range_("lbm_batch_step");
  if (!b || nsteps < 0) return LBM_EINVAL;
  if (b->ctx.empty() || nsteps == 0) return LBM_OK;
  if (b->dirty) {
    lbm_status s = batch_upload(b);
    if (s != LBM_OK) return s;
  }
  const std::vector<int> key = batch_key(b);
  int64_t left = nsteps;
  if (left >= b->chunk) {
    if (!b->graph || b->graph_key != key) {
      drop_batch_graph(b);
      hipStream_t cs;
      if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return LBM_EDEVICE;
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) e = batch_launch_steps(b, b->chunk, cs);
      hipError_t e2 = hipStreamEndCapture(cs, &g);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      (void)hipStreamDestroy(cs);
      if (e != hipSuccess) {
        b->graph = nullptr;
        return LBM_EDEVICE;
      }
      b->graph_key = key;
    }
    while (left >= b->chunk) {
      if (hipGraphLaunch(b->graph, b->stream) != hipSuccess) return LBM_EDEVICE;
      left -= b->chunk;   // even chunk: every cavity's current buffer is unchanged
    }
  }
  if (left > 0 && batch_launch_steps(b, left, b->stream) != hipSuccess) return LBM_EDEVICE;
  // buffers flipped by the remainder, per cavity as its group launched it: the populations
  // once per launch, the fields once per multi-step launch
  for (lbm_ctx *c : b->ctx) {
    const int spl = batch_ctx_spl(b, c);
    const int64_t multi = spl >= 2 ? left / spl : 0;
    const int64_t singles = left - multi * spl;
    c->step += nsteps;
    if (multi & 1) {
      c->cur ^= 1;
      c->d4cur ^= 1;
      b->dirty = true;   // parities and field buffers in the table changed
    }
    if (singles == 0) continue;
    b->dirty = true;
    if (node_walls(&c->p)) {
      // the remaining step of a node-wall cavity: its own one-step launch, on the batch's
      // stream after the group's two-step launches
      const lbm_status st = step_plain(c, singles);
      if (st != LBM_OK) return st;
    } else if (singles & 1) {
      c->cur ^= 1;
    }
  }
  return LBM_OK;
}
