// lbm_kernels.hip -- gfx950 kernels of the fused stream-and-collide step of the porous
// double-diffusive MRT lattice Boltzmann model (Liu & He, arXiv 1708.07525).
//
// One thread updates one lattice node per row of its tile:
//   pull the 9 + 5 + 5 post-collision populations of the previous level from the
//   upstream nodes (Eq. 11; walls: half-way bounce-back for f, anti-bounce-back /
//   bounce-back for g, h), form rho, T, C (Eqs. 16, 26), the buoyancy (Eq. 6), the
//   explicit velocity (Eqs. 18-19) and the total force (Eq. 5), collide f in moment
//   space (Eqs. 10, 13-15), collide g and h in moment space (Eqs. 21-25) with the source
//   term of Eq. (27) (time derivative: one-step backward difference), and store.
// Cavities whose walls pass through the boundary nodes (Eqs. 33-37, 39) have their
// perimeter nodes rebuilt by non-equilibrium extrapolation: in a one-step launch by
// work-groups of their own at its front (nee_node, the tiles skip those nodes), in the
// two-step kernel by the tiles themselves.
// The 9x9 and 5x5 transforms are written out as sums with the integer / rational
// coefficients of M, N and their inverses (the inverse of an orthogonal-row matrix is its
// transpose over the squared row norms 9, 36, 36, 6, 12, 6, 12, 4, 4 and 5, 2, 2, 20, 4).
// Populations are deviations from the rest state (rho0, T0, C0); all three storage
// types share this one node function, so results do not depend on the launch shape.
//
// One step is bound by HBM bandwidth (19 population loads + 19 stores + 4 + 4 previous-step
// field accesses + 1 porosity load per node, against ~350 flops), so there is no MFMA.  The
// one-step kernel reads each population element once, by the one node that pulls it (the
// +-1 shifted reads of neighbouring tiles hit in L2).  The two- and three-step kernels keep
// the intermediate steps of a tile and its halo in LDS, so that global memory sees about
// one step's loads and stores per launch; they visit their tiles in vertical strips (tile_of),
// so that the halo rows a tile reads from global memory are still in its XCD's L2, and FP32
// (three steps) and FP16 storage (two steps) have a taller tile for lattices that stream from
// HBM.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "lbm_internal.h"

namespace lbmk {

// ---------------------------------------------------------------- storage traits
template <typename S>
struct St;
template <>
struct St<double> {
  using R = double;
  static __device__ __forceinline__ R ld(const double *p, R) { return *p; }
  static __device__ __forceinline__ void st(double *p, R v, R) { *p = v; }
};
template <>
struct St<float> {
  using R = float;
  static __device__ __forceinline__ R ld(const float *p, R) { return *p; }
  static __device__ __forceinline__ void st(float *p, R v, R) { *p = v; }
};
template <>
struct St<_Float16> {
  using R = float;
  static __device__ __forceinline__ R ld(const _Float16 *p, R inv_scale) { return (float)(*p) * inv_scale; }
  static __device__ __forceinline__ void st(_Float16 *p, R v, R scale) { *p = (_Float16)(v * scale); }
};

template <typename R>
__device__ __forceinline__ R rsqrt_(R v);
template <>
__device__ __forceinline__ double rsqrt_(double v) { return 1.0 / sqrt(v); }
template <>
__device__ __forceinline__ float rsqrt_(float v) { return 1.0f / sqrtf(v); }

// 1/v and 1/sqrt(v) of a porosity in the porous coefficients: in FP32 the hardware
// reciprocal and reciprocal square root (1 ulp), whose error is far below the storage
// rounding of the populations; exact quotients in FP64
__device__ __forceinline__ double recip_(double v) { return 1.0 / v; }
__device__ __forceinline__ float recip_(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rsqrt_fast(double v) { return 1.0 / sqrt(v); }
__device__ __forceinline__ float rsqrt_fast(float v) { return __builtin_amdgcn_rsqf(v); }

template <typename R>
__device__ __forceinline__ R sqrt_(R v);
template <>
__device__ __forceinline__ double sqrt_(double v) { return sqrt(v); }
template <>
__device__ __forceinline__ float sqrt_(float v) { return sqrtf(v); }

// ---------------------------------------------------------------- explicit velocity
// Eqs. (18)-(19): u = v / (l0 + sqrt(l0^2 + l1 |v|)), l0 = (1 + a/2)/2, l1 = b/2, and |u|.
// In FP32 the denominator is written as 1 + e, e = a/2 + l1 |v| / (l0 + sqrt(l0^2 + l1 |v|))
// (the same number), and u = v - v e/(1 + e): 1 + e is never rounded into the result.  A
// relative bias c of the velocity solve shifts the Darcy-damped steady velocity by about c/a
// (a ~ 1e-3 per step is common), so rounding the constant l0 to FP32 (c up to 6e-8) costs
// 1e-5 - 1e-4 of the velocity after some thousand steps; this form keeps c at the size of
// the rounding of e, a ten-thousandth of that.  FP64 keeps the direct form.
// In FP32 the two quotients and the two roots use the hardware reciprocal and square root
// (1 ulp): each result only enters as a small correction (l1 |v|/(l0 + ...), e/(1 + e) ~ a/2)
// or as the speed of the Forchheimer term, so their last-bit errors shift the velocity by
// about 1e-7 of a/2 (< 1e-10 relative), far below what the 1/a amplification would show.
template <typename R>
__device__ __forceinline__ void velocity_solve(R a, R b, R vx, R vy, R &ux, R &uy, R &un) {
  const R half = R(0.5);
  const R l0 = half + R(0.25) * a;
  const R l1 = half * b;
  if constexpr (sizeof(R) == 4) {
    const R vn = __builtin_amdgcn_sqrtf(vx * vx + vy * vy);
    const R l1v = l1 * vn;
    const R e = half * a + l1v * __builtin_amdgcn_rcpf(l0 + __builtin_amdgcn_sqrtf(l0 * l0 + l1v));
    const R w = e * __builtin_amdgcn_rcpf(R(1) + e);
    ux = vx - vx * w;
    uy = vy - vy * w;
    un = vn - vn * w;
  } else {
    const R vn = sqrt_(vx * vx + vy * vy);
    const R inv_den = R(1) / (l0 + sqrt_(l0 * l0 + l1 * vn));
    ux = vx * inv_den;
    uy = vy * inv_den;
    un = vn * inv_den;
  }
}

// ---------------------------------------------------------------- collision of one node
// Inputs: the pulled deviations fd[9], gd[5], hd[5]; node porosity phi and 1/phi; the Darcy
// and Forchheimer coefficients a, b of Eq. (5); the previous-step fields (T - T0, C - C0, ux,
// uy) in prev[4].  Outputs: post-collision deviations (in place) and the fields of this level in
// prev[4], in the same form.
// SC (FP16 storage): the populations stay in the units of the power-of-two pre-scale from
// load to store, and the constants that enter the moments (rho0, T0, C0) carry the scale
// (rho0_s, T0_s, C0_s); only the fields (T - T0, C - C0 and the velocity) are formed in
// physical units.  A power of two commutes with every rounding here, so the arithmetic is that
// of physical units, scaled exactly, without a multiply per population.
template <typename R, bool SC>
__device__ __forceinline__ void collide(const Desc<R> &d, R phi, R inv_phi, R a, R b, R *fd, R *gd, R *hd,
                                        R *prev) {
  const R half = R(0.5);
  // density, momentum and scalars (Eqs. 16, 17, 26), deviation form
  const R sA = fd[1] + fd[2] + fd[3] + fd[4];
  const R sD = fd[5] + fd[6] + fd[7] + fd[8];
  const R drho = fd[0] + sA + sD;
  const R jx = (fd[1] - fd[3]) + (fd[5] - fd[6]) - (fd[7] - fd[8]);
  const R jy = (fd[2] - fd[4]) + (fd[5] + fd[6]) - (fd[7] + fd[8]);
  const R sg = gd[0] + gd[1] + gd[2] + gd[3] + gd[4];
  const R sh = hd[0] + hd[1] + hd[2] + hd[3] + hd[4];
  const R dTs = sg * d.inv_sigma;         // T - T0 (scaled with SC)
  const R dCs = sh * inv_phi;             // C - C0 (scaled with SC)
  const R dT = SC ? dTs * d.inv_scale : dTs;
  const R dC = SC ? dCs * d.inv_scale : dCs;
  // buoyancy (Eq. 6) plus any constant acceleration.  Both products are rounded before the
  // sum (no fused multiply-add), so that equal and opposite thermal and solutal terms cancel
  // exactly, as they do in Eq. (6)
  const R Gx = d.gx;
  R Gy;
  {
#pragma clang fp contract(off)
    const R bT = d.gbT * dT;
    const R bC = d.gbC * dC;
    Gy = d.gy + (bT + bC);
  }
  // explicit velocity (Eqs. 18-19), delta_t = 1
  const R vx = jx * d.inv_rho0_s + half * phi * Gx;
  const R vy = jy * d.inv_rho0_s + half * phi * Gy;
  R ux, uy, un;
  velocity_solve(a, b, vx, vy, ux, uy, un);
  const R u2 = ux * ux + uy * uy;
  // total force (Eq. 5)
  const R drag = a + b * un;
  const R Fx = phi * Gx - drag * ux;
  const R Fy = phi * Gy - drag * uy;

  // ---- D2Q9: moments m = M f (Eq. 13) of the deviations
  const R m1 = R(-4) * fd[0] - sA + R(2) * sD;
  const R m2 = R(4) * fd[0] - R(2) * sA + sD;
  const R m4 = R(-2) * (fd[1] - fd[3]) + (fd[5] - fd[6]) - (fd[7] - fd[8]);
  const R m6 = R(-2) * (fd[2] - fd[4]) + (fd[5] + fd[6]) - (fd[7] + fd[8]);
  const R m7 = (fd[1] + fd[3]) - (fd[2] + fd[4]);
  const R m8 = (fd[5] + fd[7]) - (fd[6] + fd[8]);
  // equilibrium moments (Eq. 14, alpha1 = 1, alpha2 = -3) minus those of the rest state
  const R r0 = d.rho0_s;
  const R r0p = r0 * inv_phi;
  const R e1 = R(-2) * drho + R(3) * r0p * u2;
  const R e2 = drho - R(3) * r0p * u2;
  const R jxe = r0 * ux, jye = r0 * uy;
  const R e7 = r0p * (ux * ux - uy * uy);
  const R e8 = r0p * ux * uy;
  // forcing moments (Eq. 15)
  const R S1 = R(6) * r0p * (ux * Fx + uy * Fy);
  const R S3 = r0 * Fx, S5 = r0 * Fy;
  const R S7 = R(2) * r0p * (ux * Fx - uy * Fy);
  const R S8 = r0p * (ux * Fy + uy * Fx);
  // relaxation (Eq. 10): m* = m - s (m - meq) + (1 - s/2) S
  const R p0 = drho;
  const R p1 = m1 - d.s_e * (m1 - e1) + d.k_e * S1;
  const R p2 = m2 - d.s_eps * (m2 - e2) - d.k_eps * S1;
  const R p3 = jx - d.s_j * (jx - jxe) + d.k_j * S3;
  const R p4 = m4 - d.s_q * (m4 + jxe) - d.k_q * S3;
  const R p5 = jy - d.s_j * (jy - jye) + d.k_j * S5;
  const R p6 = m6 - d.s_q * (m6 + jye) - d.k_q * S5;
  const R p7 = m7 - d.s_v * (m7 - e7) + d.k_v * S7;
  const R p8 = m8 - d.s_v * (m8 - e8) + d.k_v * S8;
  // f* = M^-1 m*
  const R a0 = p0 * R(1.0 / 9.0);
  const R a1 = p1 * R(1.0 / 36.0);
  const R a2 = p2 * R(1.0 / 36.0);
  const R a3 = p3 * R(1.0 / 6.0);
  const R a4 = p4 * R(1.0 / 12.0);
  const R a5 = p5 * R(1.0 / 6.0);
  const R a6 = p6 * R(1.0 / 12.0);
  const R a7 = p7 * R(0.25);
  const R a8 = p8 * R(0.25);
  const R axis = a0 - a1 - R(2) * a2;
  const R diag = a0 + R(2) * a1 + a2;
  fd[1] = axis + a3 - R(2) * a4 + a7;
  fd[2] = axis + a5 - R(2) * a6 - a7;
  fd[5] = diag + a3 + a4 + a5 + a6 + a8;
  fd[6] = diag - a3 - a4 + a5 + a6 - a8;
  fd[7] = diag - a3 - a4 - a5 - a6 + a8;
  fd[8] = diag + a3 + a4 - a5 - a6 - a8;
  // f3, f4 and the rest population f0 are formed from the moments they must carry
  // (sum e_x f* = m3*, sum e_y f* = m5*, sum f* = rho): algebraically the same rows of
  // M^-1, but each moment then comes back up to one rounding instead of being scaled by
  // 6 fl(1/6) or 9 fl(1/9) every step, a bias that accumulates in FP32
  fd[3] = (fd[1] + (fd[5] - fd[6])) - ((fd[7] - fd[8]) + p3);
  fd[4] = (fd[2] + (fd[5] + fd[6])) - ((fd[7] + fd[8]) + p5);
  fd[0] = drho - ((fd[1] + fd[2]) + (fd[3] + fd[4])) - ((fd[5] + fd[6]) + (fd[7] + fd[8]));

  // ---- D2Q5 for T (Eq. 21) and C (Eq. 22)
  // equilibrium fluxes T u, C u (Eqs. 24-25), formed as T0 u + (T - T0) u so that the rounding
  // of T itself does not enter; source moments N S~ = (0, d(T ux)/dt, d(T uy)/dt, 0, 0) from
  // Eq. (27) with d(T u)/dt = T0 (u - u_prev) + ((T - T0) u - (T - T0)_prev u_prev): the
  // difference of two nearly equal products T u is never formed
  const R TuX = d.T0_s * ux + dTs * ux, TuY = d.T0_s * uy + dTs * uy;
  const R CuX = d.C0_s * ux + dCs * ux, CuY = d.C0_s * uy + dCs * uy;
  const R dux = ux - prev[2], duy = uy - prev[3];
  const R pT = SC ? prev[0] * d.scale : prev[0], pC = SC ? prev[1] * d.scale : prev[1];
  const R STx = d.T0_s * dux + (dTs * ux - pT * prev[2]), STy = d.T0_s * duy + (dTs * uy - pT * prev[3]);
  const R SCx = d.C0_s * dux + (dCs * ux - pC * prev[2]), SCy = d.C0_s * duy + (dCs * uy - pC * prev[3]);
  const R kh3 = !d.phi_field ? d.kh3_u : (d.model == 0 ? (d.c5v - R(4) * phi) : (d.c5v - R(4)) * phi);
  // Both scalars collide as increments: the moment changes n* - n = -Theta (n - n^eq) +
  // (I - Theta/2) S (the conserved zeroth moment does not change), taken back to populations by
  // N^-1 and added to the pulled ones.  The rest population then gives up exactly what the other
  // four gained, measured on their rounded values, so the stored sum (sigma T, phi C) keeps its
  // value up to one rounding per step instead of one per addition of the whole populations.
  {
    const R n1 = gd[1] - gd[3], n2 = gd[2] - gd[4];
    const R n3 = R(-4) * gd[0] + gd[1] + gd[2] + gd[3] + gd[4];
    const R n4 = gd[1] - gd[2] + gd[3] - gd[4];
    const R c1 = d.k_za * STx - d.z_a * (n1 - TuX);
    const R c2 = d.k_za * STy - d.z_a * (n2 - TuY);
    const R c3 = -d.z_e * (n3 - d.kg3 * dTs);
    const R c4 = -d.z_eps * n4;
    const R a13 = R(0.05) * c3 + R(0.25) * c4, a24 = R(0.05) * c3 - R(0.25) * c4;
    const R g1 = gd[1] + (a13 + half * c1), g3 = gd[3] + (a13 - half * c1);
    const R g2 = gd[2] + (a24 + half * c2), g4 = gd[4] + (a24 - half * c2);
    gd[0] = gd[0] - (((g1 - gd[1]) + (g2 - gd[2])) + ((g3 - gd[3]) + (g4 - gd[4])));
    gd[1] = g1;
    gd[2] = g2;
    gd[3] = g3;
    gd[4] = g4;
  }
  {
    const R eD = d.e_D;
    const R n1 = hd[1] - hd[3], n2 = hd[2] - hd[4];
    const R n3 = R(-4) * hd[0] + hd[1] + hd[2] + hd[3] + hd[4];
    const R n4 = hd[1] - hd[2] + hd[3] - hd[4];
    const R c1 = d.k_eD * SCx - eD * (n1 - CuX);
    const R c2 = d.k_eD * SCy - eD * (n2 - CuY);
    const R c3 = -d.e_e * (n3 - kh3 * dCs);
    const R c4 = -d.e_eps * n4;
    const R a13 = R(0.05) * c3 + R(0.25) * c4, a24 = R(0.05) * c3 - R(0.25) * c4;
    const R h1 = hd[1] + (a13 + half * c1), h3 = hd[3] + (a13 - half * c1);
    const R h2 = hd[2] + (a24 + half * c2), h4 = hd[4] + (a24 - half * c2);
    hd[0] = hd[0] - (((h1 - hd[1]) + (h2 - hd[2])) + ((h3 - hd[3]) + (h4 - hd[4])));
    hd[1] = h1;
    hd[2] = h2;
    hd[3] = h3;
    hd[4] = h4;
  }
  prev[0] = dT;
  prev[1] = dC;
  prev[2] = ux;
  prev[3] = uy;
}

// Darcy and Forchheimer coefficients of Eq. (5) at a node, and 1/phi
template <typename R>
__device__ __forceinline__ void porous_coeffs(const Desc<R> &d, R phi, R &a, R &b, R &inv_phi) {
  if (!d.phi_field) {
    a = d.a_u;
    b = d.b_u;
    inv_phi = d.inv_phi_u;
    return;
  }
  // K = Kscale phi^3/(1-phi)^2 (Kozeny-Carman shape of Eq. 7);
  // a = phi nu/K = ca (1-phi)^2/phi^2;  Ergun F = 1.75/sqrt(150 phi^3):
  // b = phi F/sqrt(K) = cb (1-phi)/phi^2;  fixed F: b = cb (1-phi)/sqrt(phi)
  const R q = R(1) - phi;
  const R ip = recip_(phi);
  a = d.ca * q * q * ip * ip;
  b = d.ergun ? d.cb * q * ip * ip : d.cb * q * rsqrt_fast(phi);
  inv_phi = ip;
}

// ---------------------------------------------------------------- buffer memory access
// The step kernels address every plane through buffer resources: the plane offset is a
// uniform (scalar) byte offset and each lane carries one 32-bit byte offset, which keeps
// 64-bit address arithmetic out of the per-node code.  Out-of-range accesses are dropped
// by the hardware range check (loads return 0).
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;   // raw buffer, 32-bit dwords (gfx9 family)
// Cache policies of the step (gfx9 buffer instruction bit 2 = nt, non-temporal) for the
// population and the field accesses, and whether tiles are spread over the XCDs by row band.
// All three are compiled; the host picks one per launch by the bytes a step touches, the
// autotuner by timing:
//   CP_TUNED     per storage type, chosen on the 2048^2 cavity: FP32 nt loads, plain stores,
//                bands (5.89 TB/s there; 5.69 with nt stores); FP16 nt population stores,
//                plain population loads, bands (5.77); FP64 nt loads and stores in dispatch
//                order (5.56; 5.24 with bands).
//   CP_STREAM    plain loads, nt stores, bands: FP32 at other sizes (2049x2048 29.7 against
//                23.7 GLUPS with CP_TUNED, 4096^2 28.5 against 26.7).
//   CP_RESIDENT  plain loads and stores, bands: when a step touches less than the Infinity
//                Cache (256 MB) holds, the next step's reads are served from it (FP32 1024^2
//                36.0 against 27.4 GLUPS, FP64 512^2 15.6 against 13.2).
template <typename S, int CP>
struct Pol;
template <>
struct Pol<float, CP_TUNED> {
  static constexpr int load_aux = 2, store_aux = 0, fload_aux = 2, fstore_aux = 0;
  static constexpr bool xcd_bands = true;
};
template <>
struct Pol<_Float16, CP_TUNED> {
  static constexpr int load_aux = 0, store_aux = 2, fload_aux = 2, fstore_aux = 0;
  static constexpr bool xcd_bands = true;
};
template <>
struct Pol<double, CP_TUNED> {
  static constexpr int load_aux = 2, store_aux = 2, fload_aux = 2, fstore_aux = 2;
  static constexpr bool xcd_bands = false;
};
template <typename S>
struct Pol<S, CP_STREAM> {
  static constexpr int load_aux = 0, store_aux = 2, fload_aux = 0, fstore_aux = 2;
  static constexpr bool xcd_bands = true;
};
template <typename S>
struct Pol<S, CP_RESIDENT> {
  static constexpr int load_aux = 0, store_aux = 0, fload_aux = 0, fstore_aux = 0;
  static constexpr bool xcd_bands = true;
};

__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kRsrcWord3);
}

// buffer loads and stores of one element type with the cache bits LA (loads), SA (stores)
template <typename T, int LA, int SA>
struct BufIO;
template <int LA, int SA>
struct BufIO<float, LA, SA> {
  static __device__ __forceinline__ float ld(rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, LA));
  }
  static __device__ __forceinline__ void st(float x, rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, SA);
  }
};
template <int LA, int SA>
struct BufIO<double, LA, SA> {
  typedef unsigned int V2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ double ld(rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, LA));
  }
  static __device__ __forceinline__ void st(double x, rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, x), r, v, s, SA);
  }
};
template <int LA, int SA>
struct BufIO<_Float16, LA, SA> {
  static __device__ __forceinline__ _Float16 ld(rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, LA));
  }
  static __device__ __forceinline__ void st(_Float16 x, rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, SA);
  }
};
// population and field accessors of storage type S under policy CP
template <typename S, int CP>
using PopIO = BufIO<S, Pol<S, CP>::load_aux, Pol<S, CP>::store_aux>;
template <typename S, int CP>
using FieldIO = BufIO<typename St<S>::R, Pol<S, CP>::fload_aux, Pol<S, CP>::fstore_aux>;

template <typename S>
__device__ __forceinline__ typename St<S>::R to_real(S v, typename St<S>::R inv_scale);
template <>
__device__ __forceinline__ double to_real(double v, double) { return v; }
template <>
__device__ __forceinline__ float to_real(float v, float) { return v; }
// FP16 storage: the value stays in the units of the pre-scale (see collide)
template <>
__device__ __forceinline__ float to_real(_Float16 v, float) { return (float)v; }

template <typename S>
__device__ __forceinline__ S from_real(typename St<S>::R v, typename St<S>::R scale);
template <>
__device__ __forceinline__ double from_real(double v, double) { return v; }
template <>
__device__ __forceinline__ float from_real(float v, float) { return v; }
template <>
__device__ __forceinline__ _Float16 from_real(float v, float) { return (_Float16)v; }

// populations of storage type S are collided in pre-scaled units (FP16 storage)
template <typename S>
constexpr bool kScaled = __is_same(S, _Float16);

// ---------------------------------------------------------------- FP16 stochastic rounding
// Round-to-nearest binary16 storage stagnates: a population that changes by less than half a
// binary16 ulp per step never changes at all, which freezes slow diffusion.  The step kernel
// therefore rounds stochastically, with the conversion gfx950 provides for it: 13 random
// bits are added below the binary16 mantissa of the scaled binary32 value, which is then
// truncated, so the stored value is unbiased (for a binary16 subnormal result the random
// bits are aligned with the dropped bits; a value of magnitude 65504 or more goes to the
// infinity the non-finite check looks for, stochastically below 65536).  The instruction
// takes its 13 random bits from bits 19-31 of its operand.  The random bits are a function
// of (node, step, population) only, so results are reproducible and do not depend on the
// launch shape or on the other cavities of a batch: one uniform 32-bit word per node and
// step from the PCG-based hash of Jarzynski & Olano, "Hash functions for GPU rendering"
// (JCGT 2020), and for the i-th stored population of the node that word plus i times the
// 32-bit golden-ratio constant (a Weyl sequence, one addition per value).  Each value's bits
// are uniform and independent of the value, which is all the unbiased rounding needs; the
// values of one node share one draw, spread over the unit interval by the Weyl offsets.
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
  const uint32_t state = v * 747796405u + 2891336453u;
  const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}

struct Dither {
  uint32_t s;
  uint32_t k;
  __device__ __forceinline__ Dither(uint32_t node, uint32_t step) : s(pcg_hash(node ^ pcg_hash(step))), k(0) {}
  // random bits for the next population of the node (the calls come in population order)
  __device__ __forceinline__ uint32_t next13() { return s + (++k) * 0x9E3779B9u; }
};

__device__ __forceinline__ _Float16 half_stochastic(float v, uint32_t r13_hi) {
  typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
  // the conversion writes the low half and keeps the high half of its first operand, which
  // is never read: pass the random word so that no register has to be cleared for it
  return __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2_t, r13_hi), v, r13_hi, false)[0];
}

// resources of one cavity for one step
struct StepRes {
  rsrc_t src, dst, d4, phi;
};

template <typename S>
__device__ __forceinline__ StepRes step_resources(const Desc<typename St<S>::R> &d, int cur) {
  using R = typename St<S>::R;
  const uint32_t pb = (uint32_t)d.plane * (uint32_t)sizeof(S);
  const uint32_t pr = (uint32_t)d.plane * (uint32_t)sizeof(R);
  StepRes r;
  r.src = make_rsrc(cur ? d.pop1 : d.pop0, NPOP * pb);
  r.dst = make_rsrc(cur ? d.pop0 : d.pop1, NPOP * pb);
  r.d4 = make_rsrc(d.d4, ND4 * pr);
  r.phi = make_rsrc(d.phi, pr);
  return r;
}

template <typename S, int CP>
__device__ __forceinline__ void store_pop(typename St<S>::R v, typename St<S>::R scale, rsrc_t r, uint32_t voff,
                                          uint32_t soff, Dither &dz) {
  if constexpr (__is_same(S, _Float16)) {
    (void)scale;   // v is already in the units of the pre-scale
    PopIO<S, CP>::st(half_stochastic(v, dz.next13()), r, voff, soff);
  } else {
    (void)dz;
    PopIO<S, CP>::st(from_real<S>(v, scale), r, voff, soff);
  }
}

// ---------------------------------------------------------------- walls through the nodes
// Side kinds 4-7 put the wall through the first and last node of a direction.  A boundary
// node's pre-collision populations are then given by the non-equilibrium extrapolation of
// Eqs. (33)-(35) from its neighbour f along the inward normal (the inward diagonal at a
// corner):  x_b <- x^eq(b) + [x(f) - x^eq(f)], with rho_f and the wall velocity for f, and
// the boundary T, C for g, h: the side's fixed value, or Eq. (36)-(37) with zero gradient or
// with the convective gradient of Eq. (39):  T_b = (4 T_f - T_ff + 2 beta T_inf)/(3 + 2 beta),
// beta = Bi/L.  The pre-collision values of f and ff are the pulls of this same step, which
// the boundary thread recomputes from the previous level (every upstream node of f lies in
// the domain).  The boundary nodes are updated by work-groups of their own at the front of
// the step launch (nee_node); the tiles skip them, so the tile code keeps the registers and
// occupancy of the plain update.  A corner takes the rule of one of
// its sides: fixed left/right, fixed bottom/top, convective left/right, convective
// bottom/top, else zero gradient; its wall velocity is zero.
template <typename S, int CP>
__device__ __forceinline__ void pull_inner(const Desc<typename St<S>::R> &d, const StepRes &rs, int x, int y,
                                           typename St<S>::R *fd, typename St<S>::R *gd, typename St<S>::R *hd) {
  using R = typename St<S>::R;
  using IO = PopIO<S, CP>;
  constexpr uint32_t ES = sizeof(S);
  const uint32_t PB = (uint32_t)d.plane * ES;
  const int nx = d.nx, ny = d.ny, pitch = d.pitch;
  const int xm = x > 0 ? x - 1 : nx - 1, xp = x < nx - 1 ? x + 1 : 0;
  const uint32_t rm = (uint32_t)(y > 0 ? y - 1 : ny - 1) * pitch, rp = (uint32_t)(y < ny - 1 ? y + 1 : 0) * pitch;
  const uint32_t r0 = (uint32_t)y * pitch;
  const uint32_t up[9] = {r0 + x, r0 + xm, rm + x, r0 + xp, rp + x, rm + xm, rm + xp, rp + xp, rp + xm};
  const R is = d.inv_scale;
#pragma unroll
  for (int i = 0; i < 9; ++i) fd[i] = to_real<S>(IO::ld(rs.src, up[i] * ES, (uint32_t)i * PB), is);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    gd[i] = to_real<S>(IO::ld(rs.src, up[i] * ES, (uint32_t)(9 + i) * PB), is);
    hd[i] = to_real<S>(IO::ld(rs.src, up[i] * ES, (uint32_t)(14 + i) * PB), is);
  }
}

// rho - rho0, u, T - T0 and C - C0 of pre-collision populations (Eqs. 16-19, 26)
template <typename R>
__device__ __forceinline__ void node_fields(const Desc<R> &d, R phi, R a, R b, const R *fd, const R *gd, const R *hd,
                                            R &drho, R &ux, R &uy, R &dT, R &dC) {
  const R half = R(0.5);
  drho = fd[0] + (fd[1] + fd[2] + fd[3] + fd[4]) + (fd[5] + fd[6] + fd[7] + fd[8]);
  const R jx = (fd[1] - fd[3]) + (fd[5] - fd[6]) - (fd[7] - fd[8]);
  const R jy = (fd[2] - fd[4]) + (fd[5] + fd[6]) - (fd[7] + fd[8]);
  dT = (gd[0] + gd[1] + gd[2] + gd[3] + gd[4]) * d.inv_sigma;
  dC = (hd[0] + hd[1] + hd[2] + hd[3] + hd[4]) / phi;
  R Gy;
  {
#pragma clang fp contract(off)
    const R bT = d.gbT * dT;
    const R bC = d.gbC * dC;
    Gy = d.gy + (bT + bC);
  }
  const R vx = jx * d.inv_rho0 + half * phi * d.gx;
  const R vy = jy * d.inv_rho0 + half * phi * Gy;
  R un;
  velocity_solve(a, b, vx, vy, ux, uy, un);
}

// deviation-form equilibria: Eq. (20) minus w_i rho0; Eq. (28) (or the Model-A form) minus
// its value at (T0, u = 0)
template <typename R>
__device__ __forceinline__ void feq_dev(const Desc<R> &d, R drho, R ux, R uy, R phi, R *e) {
  const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const R W[9] = {R(4.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9), R(1.0 / 9),
                  R(1.0 / 36), R(1.0 / 36), R(1.0 / 36), R(1.0 / 36)};
  const R ip = R(1) / phi, u2 = ux * ux + uy * uy;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const R eu = R(EX[i]) * ux + R(EY[i]) * uy;
    e[i] = W[i] * (drho + d.rho0 * (R(3) * eu + R(4.5) * eu * eu * ip - R(1.5) * u2 * ip));
  }
}

template <typename R>
__device__ __forceinline__ void seq_dev(const Desc<R> &d, R ds, R s, R ux, R uy, R e0, R cap, R *e) {
  const R q = R(0.25) * d.varpi * cap * ds, hs = R(0.5) * s;
  e[0] = e0 * ds;
  e[1] = q + hs * ux;
  e[2] = q + hs * uy;
  e[3] = q - hs * ux;
  e[4] = q - hs * uy;
}

template <typename R>
__device__ __forceinline__ R boundary_scalar(int kind, R fixed, R beta, R amb, R sf, R sff) {
  if (kind == SIDE_NEE_HOT || kind == SIDE_NEE_COLD) return fixed;
  return (R(4) * sf - sff + R(2) * beta * amb) / (R(3) + R(2) * beta);
}

// The boundary update of node (x, y): bx / by mark a wall through the node in x / y.  Every
// load it needs (the pulls of f and ff, the porosities, the previous-step fields of the
// node) is issued before any arithmetic, so a boundary thread waits for memory once.
// pull(X, Y, f, g, h) gives the pre-collision populations of node (X, Y) of this step (from
// global memory, or from the first step's results in LDS); LOAD_PREV: read the node's
// previous-step fields into prev (else the caller has them).
template <typename S, int CP, bool LOAD_PREV, typename Pull>
__device__ __forceinline__ void nee_boundary(const Desc<typename St<S>::R> &d, const StepRes &rs, int x, int y, bool bx,
                                          bool by, typename St<S>::R *fd, typename St<S>::R *gd,
                                          typename St<S>::R *hd, typename St<S>::R *prev, typename St<S>::R &phib,
                                          Pull pull) {
  using R = typename St<S>::R;
  const int dx = bx ? (x == 0 ? 1 : -1) : 0, dy = by ? (y == 0 ? 1 : -1) : 0;
  const int sx = x == 0 ? LEFT : RIGHT, sy = y == 0 ? BOTTOM : TOP;
  // per-side values are picked with selects from uniform registers: indexing the descriptor
  // with a per-lane side would turn each into a memory round trip
  auto pick = [](auto a0, auto a1, auto a2, auto a3, int k) { return k == 0 ? a0 : k == 1 ? a1 : k == 2 ? a2 : a3; };
  const int k0 = d.kind[0], k1 = d.kind[1], k2 = d.kind[2], k3 = d.kind[3];
  int side, kind;
  R ubx = R(0), uby = R(0);
  if (bx && by) {
    const int kx = pick(k0, k1, k2, k3, sx), ky = pick(k0, k1, k2, k3, sy);
    auto fixed = [](int k) { return k == SIDE_NEE_HOT || k == SIDE_NEE_COLD; };
    side = fixed(kx) ? sx : fixed(ky) ? sy : kx == SIDE_NEE_ROBIN ? sx : ky == SIDE_NEE_ROBIN ? sy : sx;
    kind = (fixed(kx) || fixed(ky) || kx == SIDE_NEE_ROBIN || ky == SIDE_NEE_ROBIN) ? pick(k0, k1, k2, k3, side)
                                                                                    : SIDE_NEE_ADIABATIC;
  } else {
    side = bx ? sx : sy;
    kind = pick(k0, k1, k2, k3, side);
    const R uw = pick(d.uwall[0], d.uwall[1], d.uwall[2], d.uwall[3], side);
    if (bx) uby = uw;
    else ubx = uw;
  }
  const bool fixed_scalars = kind == SIDE_NEE_HOT || kind == SIDE_NEE_COLD;
  // loads: pre-collision state of f and ff (the pulls of this step), porosities, and the
  // previous-step fields of the boundary node
  const int xf = x + dx, yf = y + dy, xff = x + 2 * dx, yff = y + 2 * dy;
  const uint32_t RS = sizeof(R), PR = (uint32_t)d.plane * RS;
  const uint32_t cb = ((uint32_t)y * d.pitch + x) * RS;
  R ff[9], gf[5], hf[5], f2[9], g2[5], h2[5];
  pull(xf, yf, ff, gf, hf);
  pull(xff, yff, f2, g2, h2);
  if constexpr (kScaled<S>) {
    // the rule works in physical units; FP16 pulls carry the pre-scale
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      ff[i] *= d.inv_scale;
      f2[i] *= d.inv_scale;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      gf[i] *= d.inv_scale;
      hf[i] *= d.inv_scale;
      g2[i] *= d.inv_scale;
      h2[i] *= d.inv_scale;
    }
  }
  R phif = d.phi_u, phiff = d.phi_u;
  phib = d.phi_u;
  if (d.phi_field) {
    phib = FieldIO<S, CP>::ld(rs.phi, cb, 0);
    phif = FieldIO<S, CP>::ld(rs.phi, ((uint32_t)yf * d.pitch + xf) * RS, 0);
    phiff = FieldIO<S, CP>::ld(rs.phi, ((uint32_t)yff * d.pitch + xff) * RS, 0);
  }
  if (LOAD_PREV) {
#pragma unroll
    for (int k = 0; k < 4; ++k) prev[k] = FieldIO<S, CP>::ld(rs.d4, cb, (uint32_t)k * PR);
  }
  R af, bf, ipf;
  porous_coeffs(d, phif, af, bf, ipf);
  R drho, uxf, uyf, dTf, dCf;
  node_fields(d, phif, af, bf, ff, gf, hf, drho, uxf, uyf, dTf, dCf);
  R dTb = pick(d.Tfix[0], d.Tfix[1], d.Tfix[2], d.Tfix[3], side);
  R dCb = pick(d.Cfix[0], d.Cfix[1], d.Cfix[2], d.Cfix[3], side);
  if (!fixed_scalars) {
    const R dTff = (g2[0] + g2[1] + g2[2] + g2[3] + g2[4]) * d.inv_sigma;
    const R dCff = (h2[0] + h2[1] + h2[2] + h2[3] + h2[4]) / phiff;
    const R bT = kind == SIDE_NEE_ROBIN ? pick(d.betaT[0], d.betaT[1], d.betaT[2], d.betaT[3], side) : R(0);
    const R bC = kind == SIDE_NEE_ROBIN ? pick(d.betaC[0], d.betaC[1], d.betaC[2], d.betaC[3], side) : R(0);
    // Eq. (36) is linear, so it holds for the deviations T - T0 as well
    dTb = boundary_scalar(kind, dTb, bT, d.Tinf, dTf, dTff);
    dCb = boundary_scalar(kind, dCb, bC, d.Cinf, dCf, dCff);
  }
  R eb[9], ef[9];
  feq_dev(d, drho, ubx, uby, phib, eb);      // Eq. (33): rho of f, velocity of the wall
  feq_dev(d, drho, uxf, uyf, phif, ef);
#pragma unroll
  for (int i = 0; i < 9; ++i) fd[i] = eb[i] + (ff[i] - ef[i]);
  R sb[5], sf[5];
  seq_dev(d, dTb, d.T0 + dTb, ubx, uby, d.kg0, d.capT, sb);   // Eq. (34)
  seq_dev(d, dTf, d.T0 + dTf, uxf, uyf, d.kg0, d.capT, sf);
#pragma unroll
  for (int i = 0; i < 5; ++i) gd[i] = sb[i] + (gf[i] - sf[i]);
  const R h0b = d.model == 0 ? phib - d.varpi : (R(1) - d.varpi) * phib;
  const R h0f = d.model == 0 ? phif - d.varpi : (R(1) - d.varpi) * phif;
  seq_dev(d, dCb, d.C0 + dCb, ubx, uby, h0b, d.model == 0 ? R(1) : phib, sb);   // Eq. (35)
  seq_dev(d, dCf, d.C0 + dCf, uxf, uyf, h0f, d.model == 0 ? R(1) : phif, sf);
#pragma unroll
  for (int i = 0; i < 5; ++i) hd[i] = sb[i] + (hf[i] - sf[i]);
  if constexpr (kScaled<S>) {
#pragma unroll
    for (int i = 0; i < 9; ++i) fd[i] *= d.scale;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      gd[i] *= d.scale;
      hd[i] *= d.scale;
    }
  }
}

// Second half of a node update: collision (moment space) with the previous-step fields
// `prev` and the porous coefficients a, b (Darcy and Forchheimer terms of Eq. 5), then the
// stores.
template <typename S, int CP>
__device__ __forceinline__ void collide_store_ab(const Desc<typename St<S>::R> &d, const StepRes &rs, uint32_t c,
                                                 uint32_t step, typename St<S>::R phi, typename St<S>::R inv_phi,
                                                 typename St<S>::R a, typename St<S>::R b, typename St<S>::R *fd,
                                                 typename St<S>::R *gd, typename St<S>::R *hd,
                                                 typename St<S>::R *prev) {
  using R = typename St<S>::R;
  constexpr uint32_t ES = sizeof(S), RS = sizeof(R);
  const uint32_t PB = (uint32_t)d.plane * ES;
  const uint32_t PR = (uint32_t)d.plane * RS;
  const uint32_t cr = c * RS;
  collide<R, kScaled<S>>(d, phi, inv_phi, a, b, fd, gd, hd, prev);
  const R sc = d.scale;
  const uint32_t co = c * ES;
  Dither dz(c, step);
#pragma unroll
  for (int i = 0; i < 9; ++i) store_pop<S, CP>(fd[i], sc, rs.dst, co, (uint32_t)i * PB, dz);
#pragma unroll
  for (int i = 0; i < 5; ++i) store_pop<S, CP>(gd[i], sc, rs.dst, co, (uint32_t)(9 + i) * PB, dz);
#pragma unroll
  for (int i = 0; i < 5; ++i) store_pop<S, CP>(hd[i], sc, rs.dst, co, (uint32_t)(14 + i) * PB, dz);
  using FIO = FieldIO<S, CP>;
  FIO::st(prev[0], rs.d4, cr, 0);
  FIO::st(prev[1], rs.d4, cr, PR);
  FIO::st(prev[2], rs.d4, cr, 2 * PR);
  FIO::st(prev[3], rs.d4, cr, 3 * PR);
}

// as collide_store_ab, with the porous coefficients of Eq. (7) computed from phi
template <typename S, int CP>
__device__ __forceinline__ void collide_store(const Desc<typename St<S>::R> &d, const StepRes &rs, uint32_t c,
                                              uint32_t step, typename St<S>::R phi, typename St<S>::R *fd,
                                              typename St<S>::R *gd, typename St<S>::R *hd, typename St<S>::R *prev) {
  typename St<S>::R a, b, ip;
  porous_coeffs(d, phi, a, b, ip);
  collide_store_ab<S, CP>(d, rs, c, step, phi, ip, a, b, fd, gd, hd, prev);
}

// Second half of an interior or half-way-wall node update: previous-step fields, then
// collide_store.
template <typename S, int CP>
__device__ __forceinline__ void finish_node(const Desc<typename St<S>::R> &d, const StepRes &rs, uint32_t c,
                                            uint32_t step, typename St<S>::R phi, typename St<S>::R *fd,
                                            typename St<S>::R *gd, typename St<S>::R *hd) {
  using R = typename St<S>::R;
  const uint32_t PR = (uint32_t)d.plane * (uint32_t)sizeof(R);
  const uint32_t cr = c * (uint32_t)sizeof(R);
  R prev[4];
  using FIO = FieldIO<S, CP>;
  prev[0] = FIO::ld(rs.d4, cr, 0);
  prev[1] = FIO::ld(rs.d4, cr, PR);
  prev[2] = FIO::ld(rs.d4, cr, 2 * PR);
  prev[3] = FIO::ld(rs.d4, cr, 3 * PR);
  collide_store<S, CP>(d, rs, c, step, phi, fd, gd, hd, prev);
}

// ---------------------------------------------------------------- one node of a step
// Wall rules of a node whose links leave the domain (ok* false for a link across that side):
// f: half-way bounce-back with the moving-wall term 6 w_i rho0 e_i.u_w, the wall velocity
// tangential (along x for the bottom/top sides, along y for left/right; the axis links carry
// no tangential component); g, h: anti-bounce-back at a side held at fixed T/C, bounce-back
// at a zero-flux side.  The bounced values have already been pulled from this node.
template <typename R>
__device__ __forceinline__ void wall_rules(const Desc<R> &d, bool okxm, bool okxp, bool okym, bool okyp, R *fd,
                                           R *gd, R *hd) {
  const bool ok5 = okxm & okym, ok6 = okxp & okym, ok7 = okxp & okyp, ok8 = okxm & okyp;
  const R w5 = R(1.0 / 36.0);
  const R uB = d.uw[BOTTOM], uT = d.uw[TOP], uL = d.uw[LEFT], uR = d.uw[RIGHT];
  if (!ok5) fd[5] += w5 * (!okym ? uB : uL);
  if (!ok6) fd[6] += w5 * (!okym ? -uB : uR);
  if (!ok7) fd[7] += w5 * (!okyp ? -uT : -uR);
  if (!ok8) fd[8] += w5 * (!okyp ? uT : -uL);
  if (!okxm && d.kind[LEFT] != SIDE_ADIABATIC) {
    gd[1] = d.wT[LEFT] - gd[1];
    hd[1] = d.wC[LEFT] - hd[1];
  }
  if (!okym && d.kind[BOTTOM] != SIDE_ADIABATIC) {
    gd[2] = d.wT[BOTTOM] - gd[2];
    hd[2] = d.wC[BOTTOM] - hd[2];
  }
  if (!okxp && d.kind[RIGHT] != SIDE_ADIABATIC) {
    gd[3] = d.wT[RIGHT] - gd[3];
    hd[3] = d.wC[RIGHT] - hd[3];
  }
  if (!okyp && d.kind[TOP] != SIDE_ADIABATIC) {
    gd[4] = d.wT[TOP] - gd[4];
    hd[4] = d.wC[TOP] - hd[4];
  }
}

// Pull streaming of node (x, y) from the post-collision populations of the previous level
// in global memory (Eq. 11), with the wall rules.  INTERIOR: every upstream node lies inside
// the domain (no wall link, no wrap).
template <typename S, int CP, bool INTERIOR>
__device__ __forceinline__ void gather_global(const Desc<typename St<S>::R> &d, const StepRes &rs, int x, int y,
                                              typename St<S>::R *fd, typename St<S>::R *gd,
                                              typename St<S>::R *hd) {
  using R = typename St<S>::R;
  using IO = PopIO<S, CP>;
  constexpr uint32_t ES = sizeof(S);
  const uint32_t PB = (uint32_t)d.plane * ES;        // plane stride in bytes (populations)
  const int pitch = d.pitch, nx = d.nx, ny = d.ny;
  const uint32_t c = (uint32_t)y * pitch + x;
  bool okxm = true, okxp = true, okym = true, okyp = true;
  uint32_t xm = x - 1, xp = x + 1, rm = (uint32_t)(y - 1) * pitch, rp = (uint32_t)(y + 1) * pitch;
  if (!INTERIOR) {
    okxm = (x > 0) | d.perx;
    okxp = (x < nx - 1) | d.perx;
    okym = (y > 0) | d.pery;
    okyp = (y < ny - 1) | d.pery;
    xm = x > 0 ? x - 1 : nx - 1;
    xp = x < nx - 1 ? x + 1 : 0;
    rm = (uint32_t)(y > 0 ? y - 1 : ny - 1) * pitch;
    rp = (uint32_t)(y < ny - 1 ? y + 1 : 0) * pitch;
  }
  const uint32_t r0 = (uint32_t)y * pitch;
  const bool ok5 = okxm & okym, ok6 = okxp & okym, ok7 = okxp & okyp, ok8 = okxm & okyp;
  // byte offset of the value pulled into direction i, relative to plane min(i, opp):
  // the upstream node in plane i, or this node in plane opp(i) for a bounce-back
  auto pull = [&](bool ok, uint32_t up, int i, int o) -> uint32_t {
    const int lo = i < o ? i : o;
    const uint32_t own = c * ES + (uint32_t)(o - lo) * PB;
    const uint32_t nb = up * ES + (uint32_t)(i - lo) * PB;
    return INTERIOR ? up * ES : (ok ? nb : own);
  };
  // for INTERIOR the plane is i itself
  auto plane = [&](int i, int o) -> uint32_t { return (uint32_t)(INTERIOR ? i : (i < o ? i : o)) * PB; };
  const R is = d.inv_scale;
  const uint32_t o1 = pull(okxm, r0 + xm, 1, 3), o3 = pull(okxp, r0 + xp, 3, 1);
  const uint32_t o2 = pull(okym, rm + x, 2, 4), o4 = pull(okyp, rp + x, 4, 2);
  const uint32_t o5 = pull(ok5, rm + xm, 5, 7), o7 = pull(ok7, rp + xp, 7, 5);
  const uint32_t o6 = pull(ok6, rm + xp, 6, 8), o8 = pull(ok8, rp + xm, 8, 6);
  fd[0] = to_real<S>(IO::ld(rs.src, c * ES, 0), is);
  fd[1] = to_real<S>(IO::ld(rs.src, o1, plane(1, 3)), is);
  fd[2] = to_real<S>(IO::ld(rs.src, o2, plane(2, 4)), is);
  fd[3] = to_real<S>(IO::ld(rs.src, o3, plane(3, 1)), is);
  fd[4] = to_real<S>(IO::ld(rs.src, o4, plane(4, 2)), is);
  fd[5] = to_real<S>(IO::ld(rs.src, o5, plane(5, 7)), is);
  fd[6] = to_real<S>(IO::ld(rs.src, o6, plane(6, 8)), is);
  fd[7] = to_real<S>(IO::ld(rs.src, o7, plane(7, 5)), is);
  fd[8] = to_real<S>(IO::ld(rs.src, o8, plane(8, 6)), is);
  // g and h use the same offsets from planes 9.. and 14..
  gd[0] = to_real<S>(IO::ld(rs.src, c * ES, 9 * PB), is);
  hd[0] = to_real<S>(IO::ld(rs.src, c * ES, 14 * PB), is);
  gd[1] = to_real<S>(IO::ld(rs.src, o1, 9 * PB + plane(1, 3)), is);
  hd[1] = to_real<S>(IO::ld(rs.src, o1, 14 * PB + plane(1, 3)), is);
  gd[2] = to_real<S>(IO::ld(rs.src, o2, 9 * PB + plane(2, 4)), is);
  hd[2] = to_real<S>(IO::ld(rs.src, o2, 14 * PB + plane(2, 4)), is);
  gd[3] = to_real<S>(IO::ld(rs.src, o3, 9 * PB + plane(3, 1)), is);
  hd[3] = to_real<S>(IO::ld(rs.src, o3, 14 * PB + plane(3, 1)), is);
  gd[4] = to_real<S>(IO::ld(rs.src, o4, 9 * PB + plane(4, 2)), is);
  hd[4] = to_real<S>(IO::ld(rs.src, o4, 14 * PB + plane(4, 2)), is);
  if (!INTERIOR && !(okxm & okxp & okym & okyp)) wall_rules(d, okxm, okxp, okym, okyp, fd, gd, hd);
}

template <typename S, int CP, bool INTERIOR>
__device__ __forceinline__ void step_node(const Desc<typename St<S>::R> &d, const StepRes &rs, int x, int y,
                                          uint32_t step) {
  using R = typename St<S>::R;
  const uint32_t c = (uint32_t)y * d.pitch + x;
  R fd[9], gd[5], hd[5];
  R phi = d.phi_u;
  if (d.phi_field) phi = FieldIO<S, CP>::ld(rs.phi, c * (uint32_t)sizeof(R), 0);
  if (!INTERIOR && d.nee) {
    // walls through the nodes: the perimeter work-groups update the boundary nodes
    if ((!d.perx && (x == 0 || x == d.nx - 1)) || (!d.pery && (y == 0 || y == d.ny - 1))) return;
  }
  gather_global<S, CP, INTERIOR>(d, rs, x, y, fd, gd, hd);
  finish_node<S, CP>(d, rs, c, step, phi, fd, gd, hd);
}

// tile index -> (x0, y0), spreading consecutive row bands over the 8 XCDs so that the
// tiles that share halo cache lines run on the same XCD (work-groups are dispatched to
// XCDs round-robin by id)
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int per = n >> 3, rem = n & 7;
  const int k = b & 7, j = b >> 3;
  return k * per + (k < rem ? k : rem) + j;
}

// tile index -> tile coordinates (tx, ty) of an ntx x nty grid of tiles: row by row (sw = 0),
// or in vertical strips of sw tiles (the last one narrower when sw does not divide ntx), each
// strip walked row by row.  With the XCD bands above, the tiles an XCD runs in succession then
// lie within a strip, so the halo rows a tile reads were loaded by a tile that ran only sw
// tiles earlier and are still in that XCD's L2 (row by row, on a wide lattice they were loaded a
// whole row of tiles earlier).  A bijection for every sw >= 0.
__device__ __forceinline__ void tile_of(int b, int ntx, int nty, int sw, int &tx, int &ty) {
  if (sw <= 0 || sw >= ntx) {
    tx = b % ntx;
    ty = b / ntx;
    return;
  }
  const int st = sw * nty, s = b / st, rem = b - s * st;
  const int ws = min(sw, ntx - s * sw);
  tx = s * sw + rem % ws;
  ty = rem / ws;
}

// one tile: tile_y rows of blockDim.x nodes starting at (x0, y0)
// The tile at the origin also advances the step counter: it reads counter[cur] (the count
// of the state being read) and writes counter[cur ^ 1] (the count of the state being
// written); no other thread writes either word during the launch.
template <typename S, int CP>
__device__ __forceinline__ void step_tile(const Desc<typename St<S>::R> &d, const StepRes &rs, int cur, int x0,
                                          int y0, int tile_y) {
  const int x = x0 + threadIdx.x;
  const int y1 = min(y0 + tile_y, d.ny);
  const bool interior = x0 >= 1 && x0 + (int)blockDim.x <= d.nx - 1 && y0 >= 1 && y0 + tile_y <= d.ny - 1;
  const uint32_t step = d.counter[cur];
  if (x0 == 0 && y0 == 0 && threadIdx.x == 0) d.counter[cur ^ 1] = step + 1u;
  if (x >= d.nx) return;
  if (interior) {
    for (int y = y0; y < y1; ++y) step_node<S, CP, true>(d, rs, x, y, step);
  } else {
    for (int y = y0; y < y1; ++y) step_node<S, CP, false>(d, rs, x, y, step);
  }
}

// Boundary node k of a cavity with walls through the nodes (Eqs. 33-37, 39): the perimeter
// is numbered bottom and top rows first (when y is not periodic), then the left and right
// columns without the corners (when x is not periodic).
template <typename S, int CP>
__device__ __forceinline__ void nee_node(const Desc<typename St<S>::R> &d, const StepRes &rs, int cur, int k) {
  using R = typename St<S>::R;
  const int nx = d.nx, ny = d.ny;
  const bool wy = !d.pery, wx = !d.perx;
  const int nrow = wy ? 2 * nx : 0;
  const int h = wy ? ny - 2 : ny;
  if (k >= nrow + (wx ? 2 * h : 0)) return;
  int x, y;
  if (k < nrow) {
    x = k % nx;
    y = k < nx ? 0 : ny - 1;
  } else {
    const int q = k - nrow;
    x = q < h ? 0 : nx - 1;
    y = (wy ? 1 : 0) + q % h;
  }
  const uint32_t step = d.counter[cur];
  R fd[9], gd[5], hd[5], prev[4], phi;
  nee_boundary<S, CP, true>(d, rs, x, y, wx && (x == 0 || x == nx - 1), wy && (y == 0 || y == ny - 1), fd, gd, hd,
                            prev, phi, [&](int X, int Y, R *f, R *g, R *h) { pull_inner<S, CP>(d, rs, X, Y, f, g, h); });
  collide_store<S, CP>(d, rs, (uint32_t)y * d.pitch + x, step, phi, fd, gd, hd, prev);
}

// number of perimeter nodes nee_node covers
__host__ __device__ inline int nee_nodes(int nx, int ny, bool perx, bool pery) {
  return (pery ? 0 : 2 * nx) + (perx ? 0 : 2 * (pery ? ny : ny - 2));
}

// One time step.  The first `nperim` work-groups (a multiple of 8, zero unless the cavity
// has walls through the nodes) update the perimeter nodes, which the tiles skip; the rest
// are the tiles.  Both read only the previous level and write disjoint nodes, so the
// perimeter work overlaps the tiles within the one launch.
template <typename S, int CP>
__global__ void __launch_bounds__(256) step_kernel(const Desc<typename St<S>::R> *__restrict__ dp, int tile_y, int ntx,
                                                   int parity, int nperim) {
  // the descriptor is read from device memory as fields are needed (passed by value, all of it
  // would be loaded into scalar registers at entry and spilled)
  const Desc<typename St<S>::R> &d = *dp;
  const int cur = (d.base_parity ^ parity) & 1;
  const StepRes rs = step_resources<S>(d, cur);
  if ((int)blockIdx.x < nperim) {
    nee_node<S, CP>(d, rs, cur, (int)(blockIdx.x * blockDim.x + threadIdx.x));
    return;
  }
  const int b = (int)blockIdx.x - nperim, nb = (int)gridDim.x - nperim;
  const int t = Pol<S, CP>::xcd_bands ? xcd_remap(b, nb) : b;
  step_tile<S, CP>(d, rs, cur, (t % ntx) * blockDim.x, (t / ntx) * tile_y, tile_y);
}

// ---------------------------------------------------------------- two steps per launch
// One work-group of W x H threads advances a W x H tile by two time steps.
// Step one updates the tile and a one-node halo ((W + 2) x (H + 2) nodes, pulled from
// global memory exactly as in step_node) into LDS; step two pulls from LDS, with the same
// wall rules, and stores the tile.  Per node and two steps, global memory sees the loads of
// one step (plus the halo share, (66 x 10)/(64 x 8) = 1.29) and the stores of one step.  The
// fields of the two levels go to two buffers (d4 read, d4b written), since halo nodes are
// read by more than one work-group.  Each thread updates its own tile node in step one (one
// aligned row segment per wave, its fields kept in registers for step two) and then at most
// one node of the halo ring, so LDS holds populations only (50 KB in FP32: 3 work-groups
// per CU).  The result is bitwise that of two step_kernel launches: step one's values are
// rounded to the storage type in LDS (FP16: the same stochastic rounding with the same
// random bits) as a store and a reload would round them.
// Tile of the two-step kernel per storage type (measured, banded 2048^2 and 4096^2 cavities:
// FP32 64 x 8 51.3 GLUPS against 46.9 for 32 x 16 and 43.7 for 32 x 8; FP16 64 x 8 60.5
// against 52.2; FP64 32 x 8 24.9 against 21.8 for 32 x 16 and 22.9 for 64 x 8, its LDS being
// twice as large)
template <int W_, int H_>
struct Shape2 {
  static constexpr int W = W_, H = H_;
  static constexpr int RW = W + 2, RH = H + 2, RN = RW * RH, THREADS = W * H;
};
template <typename S>
struct TwoStepOf {
  using T = Shape2<64, 8>;
};
template <>
struct TwoStepOf<double> {
  using T = Shape2<32, 8>;
};
template <typename S>
using TwoStep = typename TwoStepOf<S>::T;
// The tile shapes a batched two-step launch may take (chosen per group by the batch
// autotuner; the first is the single-cavity tile): narrower tiles waste fewer lanes on
// cavities whose width is not a multiple of 64 (32) nodes.
template <typename S, int K>
struct BatchShape {
  using T = typename std::conditional<K == 0, Shape2<64, 8>,
                                      typename std::conditional<K == 1, Shape2<32, 16>, Shape2<32, 8>>::type>::type;
};
template <int K>
struct BatchShape<double, K> {
  using T = typename std::conditional<K == 0, Shape2<32, 8>,
                                      typename std::conditional<K == 1, Shape2<16, 16>, Shape2<16, 8>>::type>::type;
};
constexpr int kBatchShapes = 3;

template <typename S>
__device__ __forceinline__ S to_store(typename St<S>::R v, typename St<S>::R scale, Dither &dz) {
  if constexpr (__is_same(S, _Float16)) {
    (void)scale;   // v is already in the units of the pre-scale
    return half_stochastic(v, dz.next13());
  } else {
    (void)dz;
    return from_real<S>(v, scale);
  }
}

// Two steps of the tile at (x0, y0).  parity selects the population buffers as in step_kernel
// and the field buffers: read d4, write d4b when even; the other way round when odd.
// Every thread of the work-group calls this (it synchronises); none returns early.
// NEE: walls through the boundary nodes.  A boundary node takes the rule of nee_node in both
// steps, in step one from global memory, in step two from the first step's results in LDS:
// its f and ff and their upstream nodes (up to three nodes inward and one along the wall)
// lie in the tile's region, which the caller guarantees by placing the last tile of a row or
// column against the far wall (tiles then overlap and write equal values twice).
template <typename S, int CP, bool NEE, typename SH = TwoStep<S>>
__device__ __forceinline__ void two_step_tile(const Desc<typename St<S>::R> &d, int x0, int y0, int parity,
                                              S (*lpop)[SH::RN]) {
  using R = typename St<S>::R;
  using FIO = FieldIO<S, CP>;
  constexpr int TS_W = SH::W, TS_H = SH::H, TS_RW = SH::RW, TS_RH = SH::RH;
  constexpr int TS_THREADS = SH::THREADS;
  constexpr uint32_t RS = sizeof(R);
  const uint32_t PR = (uint32_t)d.plane * RS;
  const int nx = d.nx, ny = d.ny, pitch = d.pitch;
  const int cur = (d.base_parity ^ parity) & 1;
  StepRes rs = step_resources<S>(d, cur);
  const rsrc_t fread = make_rsrc((parity & 1) ? d.d4b : d.d4, ND4 * PR);
  const rsrc_t fwrite = make_rsrc((parity & 1) ? d.d4 : d.d4b, ND4 * PR);
  rs.d4 = fread;                           // the fields of step one's previous level
  const uint32_t step = d.counter[cur];
  if (x0 == 0 && y0 == 0 && threadIdx.x == 0) d.counter[cur ^ 1] = step + 2u;
  const R is = d.inv_scale, sc = d.scale;
  // the halo region and every node it pulls from lie inside the domain
  const bool interior = x0 >= 2 && x0 + TS_W + 1 <= nx - 1 && y0 >= 2 && y0 + TS_H + 1 <= ny - 1;

  // step one at region node (lx, ly) (global x0 - 1 + lx, y0 - 1 + ly): populations into
  // LDS, the fields into `prev`, the porosity and porous coefficients into `pab`
  auto step_one = [&](int lx, int ly, R *prev, R *pab) {
    int X = x0 - 1 + lx, Y = y0 - 1 + ly;
    if (!interior) {
      if (X < 0 || X >= nx) {
        if (!d.perx) return;               // outside a wall: never read in step two
        X = X < 0 ? X + nx : X - nx;
      }
      if (Y < 0 || Y >= ny) {
        if (!d.pery) return;
        Y = Y < 0 ? Y + ny : Y - ny;
      }
    }
    const uint32_t c = (uint32_t)Y * pitch + X;
    const int r = ly * TS_RW + lx;
    R fd[9], gd[5], hd[5];
    R phi = d.phi_u;
    const bool bx = NEE && !interior && !d.perx && (X == 0 || X == nx - 1);
    const bool by = NEE && !interior && !d.pery && (Y == 0 || Y == ny - 1);
    if (NEE && (bx || by)) {
      nee_boundary<S, CP, true>(d, rs, X, Y, bx, by, fd, gd, hd, prev, phi,
                                [&](int PX, int PY, R *f, R *g, R *h) { pull_inner<S, CP>(d, rs, PX, PY, f, g, h); });
    } else {
      if (d.phi_field) phi = FIO::ld(rs.phi, c * RS, 0);
      if (interior) gather_global<S, CP, true>(d, rs, X, Y, fd, gd, hd);
      else gather_global<S, CP, false>(d, rs, X, Y, fd, gd, hd);
#pragma unroll
      for (int k = 0; k < 4; ++k) prev[k] = FIO::ld(fread, c * RS, (uint32_t)k * PR);
    }
    R a, bb, ip;
    porous_coeffs(d, phi, a, bb, ip);
    pab[0] = phi;
    pab[1] = a;
    pab[2] = bb;
    pab[3] = ip;
    collide<R, kScaled<S>>(d, phi, ip, a, bb, fd, gd, hd, prev);
    Dither dz(c, step);
#pragma unroll
    for (int i = 0; i < 9; ++i) lpop[i][r] = to_store<S>(fd[i], sc, dz);
#pragma unroll
    for (int i = 0; i < 5; ++i) lpop[9 + i][r] = to_store<S>(gd[i], sc, dz);
#pragma unroll
    for (int i = 0; i < 5; ++i) lpop[14 + i][r] = to_store<S>(hd[i], sc, dz);
  };
  // each thread: its own node of the tile (fields kept in registers for step two), then at
  // most one node of the halo ring: rows ly = 0 and TS_RH - 1, then columns lx = 0 and
  // TS_RW - 1 without the corners
  const int tx = (int)threadIdx.x % TS_W, ty = (int)threadIdx.x / TS_W;
  R prev[4], pab[4];
  step_one(tx + 1, ty + 1, prev, pab);
  constexpr int NHALO = 2 * TS_RW + 2 * TS_H;
  static_assert(NHALO <= TS_THREADS, "one halo node per thread at most");
  if ((int)threadIdx.x < NHALO) {
    const int h = threadIdx.x;
    int hx, hy;
    if (h < 2 * TS_RW) {
      hx = h % TS_RW;
      hy = h < TS_RW ? 0 : TS_RH - 1;
    } else {
      const int q = h - 2 * TS_RW;
      hx = q < TS_H ? 0 : TS_RW - 1;
      hy = 1 + q % TS_H;
    }
    R unused[4], unused_pab[4];
    step_one(hx, hy, unused, unused_pab);
  }
  __syncthreads();

  // step two: the tile, pulled from LDS
  const int x = x0 + tx, y = y0 + ty;
  if (x < nx && y < ny) {
    const int r = (ty + 1) * TS_RW + tx + 1;
    const uint32_t c = (uint32_t)y * pitch + x;
    R fd[9], gd[5], hd[5];
    const bool bx = NEE && !interior && !d.perx && (x == 0 || x == nx - 1);
    const bool by = NEE && !interior && !d.pery && (y == 0 || y == ny - 1);
    auto L = [&](int pl, int off) -> R { return to_real<S>(lpop[pl][r + off], is); };
    if (NEE && (bx || by)) {
      // the pulls of f and ff from LDS (region node of (PX, PY): PX - x0 + 1, PY - y0 + 1)
      auto lds_pull = [&](int PX, int PY, R *f, R *g, R *h) {
        const int q = (PY - y0 + 1) * TS_RW + (PX - x0 + 1);
        const int up[9] = {q, q - 1, q - TS_RW, q + 1, q + TS_RW, q - TS_RW - 1, q - TS_RW + 1, q + TS_RW + 1,
                           q + TS_RW - 1};
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = to_real<S>(lpop[i][up[i]], is);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          g[i] = to_real<S>(lpop[9 + i][up[i]], is);
          h[i] = to_real<S>(lpop[14 + i][up[i]], is);
        }
      };
      R unused[4], phib;
      nee_boundary<S, CP, false>(d, rs, x, y, bx, by, fd, gd, hd, unused, phib, lds_pull);
    } else if (interior) {
      // no wall link in the tile: plain pulls
      const int off[5] = {0, -1, -TS_RW, 1, TS_RW};
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        fd[i] = L(i, off[i]);
        gd[i] = L(9 + i, off[i]);
        hd[i] = L(14 + i, off[i]);
      }
      fd[5] = L(5, -TS_RW - 1);
      fd[6] = L(6, -TS_RW + 1);
      fd[7] = L(7, TS_RW + 1);
      fd[8] = L(8, TS_RW - 1);
    } else {
      // f_i(x) = f_i*(x - e_i), or the opposite population of this node across a wall
      const bool okxm = (x > 0) | d.perx, okxp = (x < nx - 1) | d.perx;
      const bool okym = (y > 0) | d.pery, okyp = (y < ny - 1) | d.pery;
      const bool ok5 = okxm & okym, ok6 = okxp & okym, ok7 = okxp & okyp, ok8 = okxm & okyp;
      fd[0] = L(0, 0);
      fd[1] = okxm ? L(1, -1) : L(3, 0);
      fd[2] = okym ? L(2, -TS_RW) : L(4, 0);
      fd[3] = okxp ? L(3, 1) : L(1, 0);
      fd[4] = okyp ? L(4, TS_RW) : L(2, 0);
      fd[5] = ok5 ? L(5, -TS_RW - 1) : L(7, 0);
      fd[6] = ok6 ? L(6, -TS_RW + 1) : L(8, 0);
      fd[7] = ok7 ? L(7, TS_RW + 1) : L(5, 0);
      fd[8] = ok8 ? L(8, TS_RW - 1) : L(6, 0);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        R *e = q ? hd : gd;
        const int p = q ? 14 : 9;
        e[0] = L(p, 0);
        e[1] = okxm ? L(p + 1, -1) : L(p + 3, 0);
        e[2] = okym ? L(p + 2, -TS_RW) : L(p + 4, 0);
        e[3] = okxp ? L(p + 3, 1) : L(p + 1, 0);
        e[4] = okyp ? L(p + 4, TS_RW) : L(p + 2, 0);
      }
      if (!(okxm & okxp & okym & okyp)) wall_rules(d, okxm, okxp, okym, okyp, fd, gd, hd);
    }
    // the node's porosity and porous coefficients, as step one computed them (a boundary
    // node's too: the rule reads the same porosity)
    rs.d4 = fwrite;
    collide_store_ab<S, CP>(d, rs, c, step + 1u, pab[0], pab[3], pab[1], pab[2], fd, gd, hd, prev);
  }
}

// NEE: the last tile of each row and column is placed against the far side (nx >= W and
// ny >= H, checked by the launcher)
template <typename S, int CP, bool NEE, typename SH = TwoStep<S>>
__global__ void __launch_bounds__(SH::THREADS) step2_kernel(const Desc<typename St<S>::R> *__restrict__ dp, int ntx,
                                                            int parity, int sw) {
  const Desc<typename St<S>::R> &d = *dp;
  __shared__ S lpop[NPOP][SH::RN];
  const int b = Pol<S, CP>::xcd_bands ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  int tx, ty;
  tile_of(b, ntx, (int)gridDim.x / ntx, sw, tx, ty);
  int x0 = tx * SH::W, y0 = ty * SH::H;
  if (NEE) {
    x0 = min(x0, d.nx - SH::W);
    y0 = min(y0, d.ny - SH::H);
  }
  two_step_tile<S, CP, NEE, SH>(d, x0, y0, parity, lpop);
}

// The taller FP16 tile of the single-lattice two-step launch, 64 x 12 (65 VGPRs, 35 KB of LDS: two
// work-groups of 12 waves per CU), for lattices that stream from HBM.  Measured with the tiles in
// strips (banded cavity, streaming policy): 2048^2 69.5 GLUPS against 67.3 for 64 x 8 row by row,
// 4096^2 76.2 against 71.9 for 64 x 8 in strips.
using TallTwo = Shape2<64, 12>;

// ---------------------------------------------------------------- three steps per launch
// One work-group of W x H threads advances a W x H tile by three time steps (storage FP32 or
// FP64, walls half a spacing outside).  Step one updates the tile and a two-node halo
// ((W + 4) x (H + 4) nodes, pulled from global memory as in step_node) into LDS; step two
// updates the tile and the inner halo ring ((W + 2) x (H + 2) nodes) from LDS, in place: every
// thread first reads the pulls of its nodes, then, after a barrier, writes the results over
// them; step three pulls the tile from LDS and stores it.  Per node and three steps, global
// memory sees about one step's loads and one step's stores.  Each node of the region belongs
// to one thread for all its steps, so its fields and porous coefficients stay in registers:
// a thread owns its tile node, and at most one node of the inner ring (threads [0, N1)) or
// of the outer ring (threads [N1, N1 + N2)).  The values kept in LDS are rounded to the
// storage type as a store and a reload would round them, so the result is bitwise that of
// three one-step launches.
template <int W_, int H_, int MINW>
struct Shape3 {
  static constexpr int W = W_, H = H_;
  static constexpr int RW = W + 4, RH = H + 4, RN = RW * RH, THREADS = W * H;
  static constexpr int N1 = 2 * (W + 2) + 2 * H;        // inner ring
  static constexpr int N2 = 2 * RW + 2 * (H + 2);       // outer ring
  static constexpr int MIN_WAVES_PER_EU = MINW;
};
// Tiles of the batched three-step launch: those of batch tile shape 0 (FP32 64 x 8: 80 VGPRs and
// 51 KB of LDS let three work-groups of 8 waves share a CU; FP64 32 x 8)
template <typename S>
using ThreeStep = Shape3<TwoStep<S>::W, TwoStep<S>::H, sizeof(S) == 4 ? 6 : 1>;
// The taller FP32 tile of the single-lattice three-step launch, 64 x 12 (80 VGPRs, 68 KB of LDS:
// two work-groups of 12 waves per CU, 8% fewer halo collisions per stored update than 64 x 8),
// for lattices that stream from HBM.  Measured with the tiles in strips (banded cavity): 2048^2
// 67.3 GLUPS against 62.9 for 64 x 8 and 53.5 for 64 x 16 (one work-group per CU), 4096^2 74.4
// against 68.6; but 1024^2 61.1 against 65.0 and 512^2 43.5 against 48.8, where the lattice stays
// in the Infinity Cache and the third work-group per CU matters more.  Row by row 64 x 12 loses
// at 2048^2 too (58.2 against 60.2): its larger region pays once the halo rows come from the L2.
// FP64 keeps 32 x 8 (32 x 12: 26.2 against 30.7 GLUPS).
using TallThree = Shape3<64, 12, 6>;

// LDS plane of moving population i (0-8 f, 9-13 g, 14-18 h) when the rest populations f0,
// g0, h0 stay in registers: the 16 moving populations in order
__host__ __device__ constexpr int lp(int i) { return i - 1 - (i > 9 ? 1 : 0) - (i > 14 ? 1 : 0); }

template <typename S, int CP, typename TS>
__device__ __forceinline__ void three_step_tile(const Desc<typename St<S>::R> &d, int x0, int y0, int parity,
                                                S (*lpop)[TS::RN]) {
  static_assert(!kScaled<S>, "three steps per launch: FP32 and FP64 storage");
  using R = typename St<S>::R;
  using FIO = FieldIO<S, CP>;
  constexpr int W = TS::W, H = TS::H, RW = TS::RW, RH = TS::RH;
  constexpr int N1 = TS::N1, N2 = TS::N2;
  static_assert(N1 + N2 <= TS::THREADS, "one ring node per thread at most");
  constexpr uint32_t RS = sizeof(R);
  const uint32_t PR = (uint32_t)d.plane * RS;
  const int nx = d.nx, ny = d.ny, pitch = d.pitch;
  const int cur = (d.base_parity ^ parity) & 1;
  StepRes rs = step_resources<S>(d, cur);
  const rsrc_t fread = make_rsrc((parity & 1) ? d.d4b : d.d4, ND4 * PR);
  const rsrc_t fwrite = make_rsrc((parity & 1) ? d.d4 : d.d4b, ND4 * PR);
  rs.d4 = fread;
  const uint32_t step = d.counter[cur];
  if (x0 == 0 && y0 == 0 && threadIdx.x == 0) d.counter[cur ^ 1] = step + 3u;

  // the region and every node it pulls from lie inside the domain
  const bool interior = x0 >= 3 && x0 + W + 2 <= nx - 1 && y0 >= 3 && y0 + H + 2 <= ny - 1;

  // domain node of region node (lx, ly), wrapped across periodic sides; false beyond a wall
  auto locate = [&](int lx, int ly, int &X, int &Y) -> bool {
    X = x0 - 2 + lx;
    Y = y0 - 2 + ly;
    if (interior) return true;
    if (X < 0 || X >= nx) {
      if (!d.perx) return false;
      X = X < 0 ? X + nx : X - nx;
    }
    if (Y < 0 || Y >= ny) {
      if (!d.pery) return false;
      Y = Y < 0 ? Y + ny : Y - ny;
    }
    return true;
  };
  // the rest populations f0, g0, h0 are pulled only by their own node, whose thread keeps
  // them in registers (rest[3]); LDS holds the 16 moving populations (plane lp(i))
  auto lds_store = [&](int r, const R *fd, const R *gd, const R *hd, R *rest) {
#pragma unroll
    for (int i = 1; i < 9; ++i) lpop[lp(i)][r] = (S)fd[i];
#pragma unroll
    for (int i = 1; i < 5; ++i) lpop[lp(9 + i)][r] = (S)gd[i];
#pragma unroll
    for (int i = 1; i < 5; ++i) lpop[lp(14 + i)][r] = (S)hd[i];
    rest[0] = fd[0];
    rest[1] = gd[0];
    rest[2] = hd[0];
  };
  // step one at region node (lx, ly): populations into LDS, fields into prev, porosity and
  // porous coefficients into pab
  auto step_one = [&](int lx, int ly, R *prev, R *pab, R *rest) {
    int X, Y;
    if (!locate(lx, ly, X, Y)) return;     // beyond a wall: never read
    const uint32_t c = (uint32_t)Y * pitch + X;
    R fd[9], gd[5], hd[5];
    R phi = d.phi_u;
    if (d.phi_field) phi = FIO::ld(rs.phi, c * RS, 0);
    if (interior) gather_global<S, CP, true>(d, rs, X, Y, fd, gd, hd);
    else gather_global<S, CP, false>(d, rs, X, Y, fd, gd, hd);
#pragma unroll
    for (int k = 0; k < 4; ++k) prev[k] = FIO::ld(fread, c * RS, (uint32_t)k * PR);
    R a, bb, ip;
    porous_coeffs(d, phi, a, bb, ip);
    pab[0] = phi;
    pab[1] = a;
    pab[2] = bb;
    pab[3] = ip;
    collide<R, kScaled<S>>(d, phi, ip, a, bb, fd, gd, hd, prev);
    lds_store(ly * RW + lx, fd, gd, hd, rest);
  };
  // pulls of region node (lx, ly) = domain node (X, Y) from LDS, with the wall rules
  auto lds_pulls = [&](int lx, int ly, int X, int Y, R *fd, R *gd, R *hd, const R *rest) {
    const int r = ly * RW + lx;
    auto L = [&](int pl, int off) -> R { return (R)lpop[lp(pl)][r + off]; };
    fd[0] = rest[0];
    gd[0] = rest[1];
    hd[0] = rest[2];
    if (interior) {
      const int off[5] = {0, -1, -RW, 1, RW};
#pragma unroll
      for (int i = 1; i < 5; ++i) {
        fd[i] = L(i, off[i]);
        gd[i] = L(9 + i, off[i]);
        hd[i] = L(14 + i, off[i]);
      }
      fd[5] = L(5, -RW - 1);
      fd[6] = L(6, -RW + 1);
      fd[7] = L(7, RW + 1);
      fd[8] = L(8, RW - 1);
      return;
    }
    const bool okxm = (X > 0) | d.perx, okxp = (X < nx - 1) | d.perx;
    const bool okym = (Y > 0) | d.pery, okyp = (Y < ny - 1) | d.pery;
    const bool ok5 = okxm & okym, ok6 = okxp & okym, ok7 = okxp & okyp, ok8 = okxm & okyp;
    fd[1] = okxm ? L(1, -1) : L(3, 0);
    fd[2] = okym ? L(2, -RW) : L(4, 0);
    fd[3] = okxp ? L(3, 1) : L(1, 0);
    fd[4] = okyp ? L(4, RW) : L(2, 0);
    fd[5] = ok5 ? L(5, -RW - 1) : L(7, 0);
    fd[6] = ok6 ? L(6, -RW + 1) : L(8, 0);
    fd[7] = ok7 ? L(7, RW + 1) : L(5, 0);
    fd[8] = ok8 ? L(8, RW - 1) : L(6, 0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      R *e = q ? hd : gd;
      const int p = q ? 14 : 9;
      e[1] = okxm ? L(p + 1, -1) : L(p + 3, 0);
      e[2] = okym ? L(p + 2, -RW) : L(p + 4, 0);
      e[3] = okxp ? L(p + 3, 1) : L(p + 1, 0);
      e[4] = okyp ? L(p + 4, RW) : L(p + 2, 0);
    }
    if (!(okxm & okxp & okym & okyp)) wall_rules(d, okxm, okxp, okym, okyp, fd, gd, hd);
  };

  const int t = (int)threadIdx.x;
  const int tx = t % W, ty = t / W;
  // this thread's ring node: inner ring (rows 1 and RH - 2, then columns 1 and RW - 2), or
  // outer ring (rows 0 and RH - 1, then columns 0 and RW - 1)
  int rx = 0, ry = 0;
  const bool ring1 = t < N1, ring2 = t >= N1 && t < N1 + N2;
  if (ring1) {
    if (t < 2 * (W + 2)) {
      rx = 1 + t % (W + 2);
      ry = t < W + 2 ? 1 : RH - 2;
    } else {
      const int q = t - 2 * (W + 2);
      rx = q < H ? 1 : RW - 2;
      ry = 2 + q % H;
    }
  } else if (ring2) {
    const int k = t - N1;
    if (k < 2 * RW) {
      rx = k % RW;
      ry = k < RW ? 0 : RH - 1;
    } else {
      const int q = k - 2 * RW;
      rx = q < H + 2 ? 0 : RW - 1;
      ry = 1 + q % (H + 2);
    }
  }

  // step one: own node, then the ring node
  R prev[4], pab[4], prev1[4], pab1[4], rest[3], rest1[3];
  step_one(tx + 2, ty + 2, prev, pab, rest);
  if (ring1 || ring2) step_one(rx, ry, prev1, pab1, rest1);
  __syncthreads();

  // step two, in place: read the pulls of the own node and of an inner-ring node, then write.
  // Every region node step one computed is updated (across a periodic side a ragged tile's
  // own positions past the edge hold wrapped nodes, which step three pulls from)
  int X, Y, X1 = 0, Y1 = 0;
  const bool own_in = locate(tx + 2, ty + 2, X, Y);
  const bool r1_in = ring1 && locate(rx, ry, X1, Y1);
  R fd[9], gd[5], hd[5], f1[9], g1[5], h1[5];
  if (own_in) lds_pulls(tx + 2, ty + 2, X, Y, fd, gd, hd, rest);
  if (r1_in) lds_pulls(rx, ry, X1, Y1, f1, g1, h1, rest1);
  __syncthreads();
  if (own_in) {
    collide<R, kScaled<S>>(d, pab[0], pab[3], pab[1], pab[2], fd, gd, hd, prev);
    lds_store((ty + 2) * RW + tx + 2, fd, gd, hd, rest);
  }
  if (r1_in) {
    collide<R, kScaled<S>>(d, pab1[0], pab1[3], pab1[1], pab1[2], f1, g1, h1, prev1);
    lds_store(ry * RW + rx, f1, g1, h1, rest1);
  }
  __syncthreads();

  // step three: the tile's nodes inside the domain, pulled from LDS, stored to global memory
  if (x0 + tx < nx && y0 + ty < ny) {
    lds_pulls(tx + 2, ty + 2, X, Y, fd, gd, hd, rest);
    rs.d4 = fwrite;
    collide_store_ab<S, CP>(d, rs, (uint32_t)Y * pitch + X, step + 2u, pab[0], pab[3], pab[1], pab[2], fd, gd, hd,
                            prev);
  }
}

template <typename S, int CP, typename TS>
__global__ void __launch_bounds__(TS::THREADS, TS::MIN_WAVES_PER_EU) step3_kernel(const Desc<typename St<S>::R> *__restrict__ dp,
                                                                      int ntx, int parity, int sw) {
  const Desc<typename St<S>::R> &d = *dp;
  __shared__ S lpop[NPOP - 3][TS::RN];
  const int b = Pol<S, CP>::xcd_bands ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  int tx, ty;
  tile_of(b, ntx, (int)gridDim.x / ntx, sw, tx, ty);
  three_step_tile<S, CP, TS>(d, tx * TS::W, ty * TS::H, parity, lpop);
}

// Batched two steps over items of W x H tiles (item.tw = W, the group's shape SH): one item per
// work-group (a loop over items keeps values live across iterations and costs a third of the
// occupancy); the grid may exceed the item count, the extra work-groups exit at once.
template <typename S, int CP, typename SH>
__global__ void __launch_bounds__(SH::THREADS) step2_batch_kernel(const Desc<typename St<S>::R> *__restrict__ descs,
                                                                  const Item *__restrict__ items,
                                                                  const int *__restrict__ range, int parity) {
  __shared__ S lpop[NPOP][SH::RN];
  const int first = range[0], n = range[1];
  if ((int)blockIdx.x >= n) return;
  const int it = Pol<S, CP>::xcd_bands ? xcd_remap(blockIdx.x, n) : (int)blockIdx.x;
  const Item item = items[first + it];
  two_step_tile<S, CP, false, SH>(descs[item.cavity], item.x0, item.y0, parity, lpop);
}

// Batched two steps with walls through the boundary nodes (FP32, FP64): items of two-step tiles
// placed as step2_kernel places them (the last tile of a row or column against the far wall),
// one item per work-group.
template <typename S, int CP>
__global__ void __launch_bounds__(TwoStep<S>::THREADS)
    step2_batch_nee_kernel(const Desc<typename St<S>::R> *__restrict__ descs, const Item *__restrict__ items,
                           const int *__restrict__ range, int parity) {
  __shared__ S lpop[NPOP][TwoStep<S>::RN];
  const int first = range[0], n = range[1];
  if ((int)blockIdx.x >= n) return;
  const int it = Pol<S, CP>::xcd_bands ? xcd_remap(blockIdx.x, n) : (int)blockIdx.x;
  const Item item = items[first + it];
  two_step_tile<S, CP, true>(descs[item.cavity], item.x0, item.y0, parity, lpop);
}

// Batched three steps over items of ThreeStep<S> tiles (FP32, FP64): one item per work-group,
// as step2_batch_kernel.
template <typename S, int CP>
__global__ void __launch_bounds__(ThreeStep<S>::THREADS, ThreeStep<S>::MIN_WAVES_PER_EU)
    step3_batch_kernel(const Desc<typename St<S>::R> *__restrict__ descs, const Item *__restrict__ items,
                       const int *__restrict__ range, int parity) {
  __shared__ S lpop[NPOP - 3][ThreeStep<S>::RN];
  const int first = range[0], n = range[1];
  if ((int)blockIdx.x >= n) return;
  const int it = Pol<S, CP>::xcd_bands ? xcd_remap(blockIdx.x, n) : (int)blockIdx.x;
  const Item item = items[first + it];
  three_step_tile<S, CP, ThreeStep<S>>(descs[item.cavity], item.x0, item.y0, parity, lpop);
}

// A 256-thread tile of tw x (256/tw) nodes (tw = 64, 128 or 256), so that narrow cavities
// keep every lane busy.
template <typename S, int CP>
__device__ __forceinline__ void step_tile2d(const Desc<typename St<S>::R> &d, const StepRes &rs, int cur, int x0,
                                            int y0, int tw) {
  const int rows = (int)blockDim.x / tw;
  const int x = x0 + ((int)threadIdx.x & (tw - 1));
  const int y = y0 + (int)threadIdx.x / tw;
  const bool interior = x0 >= 1 && x0 + tw <= d.nx - 1 && y0 >= 1 && y0 + rows <= d.ny - 1;
  const uint32_t step = d.counter[cur];
  if (x0 == 0 && y0 == 0 && threadIdx.x == 0) d.counter[cur ^ 1] = step + 1u;
  if (x >= d.nx || y >= d.ny) return;
  if (interior)
    step_node<S, CP, true>(d, rs, x, y, step);
  else
    step_node<S, CP, false>(d, rs, x, y, step);
}

// Batched step: a fixed grid walks the (cavity, tile) work items of one group of attached
// cavities, items [range[0], range[0] + range[1]) of the table; the range lives in device
// memory so the host can change the batch between graph replays without re-capturing.
// Each work-group takes a contiguous run of items
// (neighbouring tiles of one cavity, so shared halo lines stay in its L2), and runs are
// laid out over the XCDs in bands as in the single-cavity kernel.  Cavities with walls
// through the boundary nodes are not batched (the host refuses to attach them).
template <typename S, int CP>
__global__ void __launch_bounds__(256) step_batch_kernel(const Desc<typename St<S>::R> *__restrict__ descs,
                                                         const Item *__restrict__ items,
                                                         const int *__restrict__ range, int parity) {
  const int first = range[0], n = range[1];
  const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
  const int b = Pol<S, CP>::xcd_bands ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int end = min(n, (b + 1) * per);
  for (int it = b * per; it < end; ++it) {
    const Item item = items[first + it];
    const Desc<typename St<S>::R> &d = descs[item.cavity];
    const int cur = (d.base_parity ^ parity) & 1;
    StepRes rs = step_resources<S>(d, cur);
    // bit 1 of parity: the fields are in the second buffer (after an odd number of two-step
    // launches of the same replay)
    if (parity & 2) rs.d4 = make_rsrc(d.d4b, ND4 * (uint32_t)d.plane * (uint32_t)sizeof(typename St<S>::R));
    step_tile2d<S, CP>(d, rs, cur, item.x0, item.y0, item.tw);
  }
}

// ---------------------------------------------------------------- initial state
// Equilibria of Eqs. (20) and (28) with rho = rho0 and the given T, C, u (deviation
// form, evaluated in FP64), then one collision; writes buffer 0 and the fields of level 0.
template <typename S>
__global__ void __launch_bounds__(256) init_kernel(Desc<typename St<S>::R> d, const double *__restrict__ Tin,
                                                   const double *__restrict__ Cin,
                                                   const double *__restrict__ uxin,
                                                   const double *__restrict__ uyin) {
  using R = typename St<S>::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= d.nx) return;
  const long long k = (long long)y * d.nx + x;
  const long long c = (long long)y * d.pitch + x;
  const long long P = d.plane;
  const double T = Tin[k], C = Cin[k], ux = uxin[k], uy = uyin[k];
  const double phi = d.phi_field ? (double)((const R *)d.phi)[c] : (double)d.phi_u;
  const double rho0 = d.rho0, varpi = d.varpi;
  const double dT = T - (double)d.T0, dC = C - (double)d.C0;
  const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  R fd[9], gd[5], hd[5], prev[4];
  const double u2 = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    const double eu = EX[i] * ux + EY[i] * uy;
    fd[i] = (R)(W[i] * rho0 * (3.0 * eu + 4.5 * eu * eu / phi - 1.5 * u2 / phi));
  }
  const double capT = d.model == 0 ? 1.0 : (double)d.sigma;
  const double capC = d.model == 0 ? 1.0 : phi;
  gd[0] = (R)(d.model == 0 ? ((double)d.sigma - varpi) * dT : (1.0 - varpi) * (double)d.sigma * dT);
  hd[0] = (R)(d.model == 0 ? (phi - varpi) * dC : (1.0 - varpi) * phi * dC);
  for (int i = 1; i < 5; ++i) {
    const double eu = EX[i] * ux + EY[i] * uy;
    gd[i] = (R)(0.25 * varpi * capT * dT + 0.5 * T * eu);
    hd[i] = (R)(0.25 * varpi * capC * dC + 0.5 * C * eu);
  }
  prev[0] = (R)dT;
  prev[1] = (R)dC;
  prev[2] = (R)ux;
  prev[3] = (R)uy;
  // the stored populations of level 0 are rounded to the storage type before colliding,
  // exactly as a pulled value would be (FP16: in the units of the pre-scale, as the step
  // kernels collide them)
  const R is = d.inv_scale, sc = d.scale;
  auto rnd = [&](R v) -> R { return to_real<S>(from_real<S>(kScaled<S> ? v * sc : v, sc), is); };
  for (int i = 0; i < 9; ++i) fd[i] = rnd(fd[i]);
  for (int i = 0; i < 5; ++i) gd[i] = rnd(gd[i]);
  for (int i = 0; i < 5; ++i) hd[i] = rnd(hd[i]);
  R a, b, ip;
  porous_coeffs(d, (R)phi, a, b, ip);
  collide<R, kScaled<S>>(d, (R)phi, ip, a, b, fd, gd, hd, prev);
  S *dst = (S *)(d.base_parity ? d.pop1 : d.pop0);
  for (int i = 0; i < 9; ++i) dst[i * P + c] = from_real<S>(fd[i], sc);
  for (int i = 0; i < 5; ++i) dst[(9 + i) * P + c] = from_real<S>(gd[i], sc);
  for (int i = 0; i < 5; ++i) dst[(14 + i) * P + c] = from_real<S>(hd[i], sc);
  R *d4 = (R *)d.d4;
  d4[c] = prev[0];
  d4[P + c] = prev[1];
  d4[2 * P + c] = prev[2];
  d4[3 * P + c] = prev[3];
}

// ---------------------------------------------------------------- reductions
// FP64 accumulation in a fixed order: thread t of block b always handles the same nodes,
// waves reduce with lane shuffles, blocks combine their waves in lane order, and one
// block combines the block partials in index order.
constexpr int OBS_ROWS = 4;
constexpr int OBS_THREADS = 256;
constexpr int NSLOT = 12;   // mass heat solute du2 u2 dT2 T2 dC2 C2 max_ux max_uy nonfinite

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <typename S>
__global__ void __launch_bounds__(OBS_THREADS) obs_partial_kernel(Desc<typename St<S>::R> d, int parity,
                                                                  typename St<S>::R *__restrict__ snap,
                                                                  double *__restrict__ partials) {
  using R = typename St<S>::R;
  const long long P = d.plane;
  const int cur = (d.base_parity ^ parity) & 1;
  const S *pop = (const S *)(cur ? d.pop1 : d.pop0);
  const R *d4 = (const R *)d.d4;
  double acc[NSLOT];
  for (int s = 0; s < NSLOT; ++s) acc[s] = 0.0;
  const int y0 = blockIdx.x * OBS_ROWS;
  const int y1 = min(y0 + OBS_ROWS, d.ny);
  for (int y = y0; y < y1; ++y) {
    for (int x = threadIdx.x; x < d.nx; x += OBS_THREADS) {
      const long long c = (long long)y * d.pitch + x;
      double drho = 0.0;
      for (int i = 0; i < 9; ++i) drho += (double)St<S>::ld(pop + i * P + c, d.inv_scale);
      const double rho = (double)d.rho0 + drho;
      // the field buffer holds T - T0 and C - C0
      const double dT = d4[c], dC = d4[P + c], ux = d4[2 * P + c], uy = d4[3 * P + c];
      const double T = (double)d.T0 + dT, C = (double)d.C0 + dC;
      const double phi = d.phi_field ? (double)((const R *)d.phi)[c] : (double)d.phi_u;
      acc[0] += rho;
      acc[1] += (double)d.sigma * T;
      acc[2] += phi * C;
      const double sT = snap[c], sC = snap[P + c], sx = snap[2 * P + c], sy = snap[3 * P + c];   // deviations
      acc[3] += (ux - sx) * (ux - sx) + (uy - sy) * (uy - sy);
      acc[4] += ux * ux + uy * uy;
      acc[5] += (dT - sT) * (dT - sT);
      acc[6] += T * T;
      acc[7] += (dC - sC) * (dC - sC);
      acc[8] += C * C;
      acc[9] = fmax(acc[9], fabs(ux));
      acc[10] = fmax(acc[10], fabs(uy));
      const bool bad = !(isfinite(rho) && isfinite(T) && isfinite(C) && isfinite(ux) && isfinite(uy));
      acc[11] += bad ? 1.0 : 0.0;
      snap[c] = (R)dT;
      snap[P + c] = (R)dC;
      snap[2 * P + c] = (R)ux;
      snap[3 * P + c] = (R)uy;
    }
  }
  __shared__ double red[OBS_THREADS / 64][NSLOT];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int s = 0; s < NSLOT; ++s) {
    const double v = (s == 9 || s == 10) ? wave_max(acc[s]) : wave_sum(acc[s]);
    if (lane == 0) red[wv][s] = v;
  }
  __syncthreads();
  if (threadIdx.x < NSLOT) {
    const int s = threadIdx.x;
    double v = red[0][s];
    for (int w = 1; w < OBS_THREADS / 64; ++w) v = (s == 9 || s == 10) ? fmax(v, red[w][s]) : v + red[w][s];
    partials[(long long)blockIdx.x * NSLOT + s] = v;
  }
}

// Mean Nusselt / Sherwood numbers of Eq. (38) at the four sides; one block per side.
// Half-way wall: gradient along the inward normal (-8 s_w + 9 s_0 - s_1)/3, mean over the
// nodes.  Wall through the nodes: (-3 s_b + 4 s_1 - s_2)/2, trapezoidal mean along the wall.
// Both stencils sum to zero, so they act on the stored deviations T - T0, C - C0 (wT, wC: the
// wall values minus T0, C0) unchanged.
// Heat entering through a hot side or leaving through a cold or convective side is positive.
template <typename R>
__global__ void __launch_bounds__(256) wall_kernel(Desc<R> d, const double *__restrict__ wT,
                                                   const double *__restrict__ wC, double LdT, double LdC,
                                                   double *__restrict__ out) {
  const int side = blockIdx.x;
  const R *d4 = (const R *)d.d4;
  const long long P = d.plane;
  const int kind = d.kind[side];
  const bool half = kind == SIDE_HOT || kind == SIDE_COLD;
  const bool node = kind == SIDE_NEE_HOT || kind == SIDE_NEE_COLD || kind == SIDE_NEE_ROBIN;
  const int n_along = (side == LEFT || side == RIGHT) ? d.ny : d.nx;
  const long long step_in = (side == LEFT) ? 1 : (side == RIGHT) ? -1 : (side == BOTTOM) ? d.pitch : -(long long)d.pitch;
  double sT = 0.0, sC = 0.0;
  if (half || node) {
    for (int a = threadIdx.x; a < n_along; a += blockDim.x) {
      long long k0;
      if (side == LEFT) k0 = (long long)a * d.pitch;
      else if (side == RIGHT) k0 = (long long)a * d.pitch + d.nx - 1;
      else if (side == BOTTOM) k0 = a;
      else k0 = (long long)(d.ny - 1) * d.pitch + a;
      const long long k1 = k0 + step_in, k2 = k0 + 2 * step_in;
      if (half) {
        sT += (-8.0 * wT[side] + 9.0 * (double)d4[k0] - (double)d4[k1]) / 3.0;
        sC += (-8.0 * wC[side] + 9.0 * (double)d4[P + k0] - (double)d4[P + k1]) / 3.0;
      } else {
        const double w = (a == 0 || a == n_along - 1) ? 0.5 : 1.0;
        sT += w * (-3.0 * (double)d4[k0] + 4.0 * (double)d4[k1] - (double)d4[k2]) / 2.0;
        sC += w * (-3.0 * (double)d4[P + k0] + 4.0 * (double)d4[P + k1] - (double)d4[P + k2]) / 2.0;
      }
    }
  }
  __shared__ double red[2][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  sT = wave_sum(sT);
  sC = wave_sum(sC);
  if (lane == 0) { red[0][wv] = sT; red[1][wv] = sC; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double aT = 0.0, aC = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { aT += red[0][w]; aC += red[1][w]; }
    const double sign = (kind == SIDE_HOT || kind == SIDE_NEE_HOT) ? -1.0 : 1.0;
    const double n = half ? (double)n_along : (double)(n_along - 1);
    out[NSLOT + side] = (half || node) ? sign * LdT * aT / n : 0.0;
    out[NSLOT + 4 + side] = (half || node) ? sign * LdC * aC / n : 0.0;
  }
}

// One work-group per slot: thread t combines the partials t, t + 256, ... in index order, then
// the waves reduce with lane shuffles and the four wave results are combined in wave order (a
// fixed tree: the result depends on the number of partials only).
__global__ void __launch_bounds__(OBS_THREADS) obs_final_kernel(const double *__restrict__ partials, int nblocks,
                                                                double *__restrict__ out) {
  const int s = blockIdx.x;
  const bool is_max = s == 9 || s == 10;
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += OBS_THREADS) {
    const double p = partials[(long long)b * NSLOT + s];
    v = is_max ? fmax(v, p) : v + p;
  }
  v = is_max ? wave_max(v) : wave_sum(v);
  __shared__ double red[OBS_THREADS / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < OBS_THREADS / 64; ++w) r = is_max ? fmax(r, red[w]) : r + red[w];
    out[s] = r;
  }
}

// FP64 fields rho, ux, uy, T, C of the current level (5 planes of nx*ny, x fastest)
template <typename S>
__global__ void __launch_bounds__(256) export_kernel(Desc<typename St<S>::R> d, int parity,
                                                     double *__restrict__ f) {
  using R = typename St<S>::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= d.nx) return;
  const long long P = d.plane, c = (long long)y * d.pitch + x;
  const long long n = (long long)d.nx * d.ny, k = (long long)y * d.nx + x;
  const int cur = (d.base_parity ^ parity) & 1;
  const S *pop = (const S *)(cur ? d.pop1 : d.pop0);
  const R *d4 = (const R *)d.d4;
  double drho = 0.0;
  for (int i = 0; i < 9; ++i) drho += (double)St<S>::ld(pop + i * P + c, d.inv_scale);
  f[k] = (double)d.rho0 + drho;
  f[n + k] = d4[2 * P + c];
  f[2 * n + k] = d4[3 * P + c];
  f[3 * n + k] = (double)d.T0 + d4[c];
  f[4 * n + k] = (double)d.C0 + d4[P + c];
}

// ---------------------------------------------------------------- launchers
template <typename S>
static int init_t(const void *desc, const double *T, const double *C, const double *ux, const double *uy,
                  void *stream) {
  const auto &d = *(const Desc<typename St<S>::R> *)desc;
  dim3 grid((d.nx + 255) / 256, d.ny);
  hipLaunchKernelGGL(init_kernel<S>, grid, dim3(256), 0, (hipStream_t)stream, d, T, C, ux, uy);
  return (int)hipGetLastError();
}

int launch_init(int prec, const void *desc, const double *T, const double *C, const double *ux,
                const double *uy, void *stream) {
  switch (prec) {
    case PREC_FP64: return init_t<double>(desc, T, C, ux, uy, stream);
    case PREC_FP32: return init_t<float>(desc, T, C, ux, uy, stream);
    default: return init_t<_Float16>(desc, T, C, ux, uy, stream);
  }
}

template <typename S, int CP>
static void step_cp(const Desc<typename St<S>::R> &d, const void *ddev, Tile tile, int parity, hipStream_t stream) {
  // with walls through the nodes the last column / row is perimeter work: the tiles need
  // only cover [0, n - 1) (node 0 is skipped inside its tile)
  const int ex = d.nee && !d.perx ? 1 : 0, ey = d.nee && !d.pery ? 1 : 0;
  const int ntx = (d.nx - ex + tile.tx - 1) / tile.tx;
  const int nty = (d.ny - ey + tile.ty - 1) / tile.ty;
  int nperim = 0;
  if (d.nee) nperim = ((nee_nodes(d.nx, d.ny, d.perx != 0, d.pery != 0) + tile.tx - 1) / tile.tx + 7) / 8 * 8;
  hipLaunchKernelGGL((step_kernel<S, CP>), dim3(nperim + ntx * nty), dim3(tile.tx), 0, stream,
                     (const Desc<typename St<S>::R> *)ddev, tile.ty, ntx, parity, nperim);
}

template <typename S>
static int step_t(const void *desc, const void *ddev, Tile tile, int cp, int parity, void *stream) {
  const auto &d = *(const Desc<typename St<S>::R> *)desc;
  hipStream_t s = (hipStream_t)stream;
  switch (cp) {
    case CP_STREAM: step_cp<S, CP_STREAM>(d, ddev, tile, parity, s); break;
    case CP_RESIDENT: step_cp<S, CP_RESIDENT>(d, ddev, tile, parity, s); break;
    default: step_cp<S, CP_TUNED>(d, ddev, tile, parity, s); break;
  }
  return (int)hipGetLastError();
}

int launch_step(int prec, const void *desc, const void *ddev, Tile tile, int cp, int parity, void *stream) {
  switch (prec) {
    case PREC_FP64: return step_t<double>(desc, ddev, tile, cp, parity, stream);
    case PREC_FP32: return step_t<float>(desc, ddev, tile, cp, parity, stream);
    default: return step_t<_Float16>(desc, ddev, tile, cp, parity, stream);
  }
}

template <typename S, typename SH = TwoStep<S>>
static int step2_t(const void *desc, const void *ddev, int cp, int parity, int sw, void *stream) {
  const auto &d = *(const Desc<typename St<S>::R> *)desc;
  const auto *dp = (const Desc<typename St<S>::R> *)ddev;
  hipStream_t s = (hipStream_t)stream;
  constexpr int W = SH::W, H = SH::H;
  const int ntx = (d.nx + W - 1) / W, nty = (d.ny + H - 1) / H;
  const dim3 grid(ntx * nty), block(SH::THREADS);
  if (d.nee) {
    // FP16 storage with walls through the nodes runs one step per launch; the tiles placed
    // against the far sides must fit in the lattice
    if constexpr (__is_same(S, _Float16)) {
      return (int)hipErrorInvalidValue;
    } else {
      if (d.nx < W || d.ny < H) return (int)hipErrorInvalidValue;
      switch (cp) {
        case CP_STREAM:
          hipLaunchKernelGGL((step2_kernel<S, CP_STREAM, true, SH>), grid, block, 0, s, dp, ntx, parity, sw);
          break;
        case CP_RESIDENT:
          hipLaunchKernelGGL((step2_kernel<S, CP_RESIDENT, true, SH>), grid, block, 0, s, dp, ntx, parity, sw);
          break;
        default:
          hipLaunchKernelGGL((step2_kernel<S, CP_TUNED, true, SH>), grid, block, 0, s, dp, ntx, parity, sw);
          break;
      }
      return (int)hipGetLastError();
    }
  }
  switch (cp) {
    case CP_STREAM:
      hipLaunchKernelGGL((step2_kernel<S, CP_STREAM, false, SH>), grid, block, 0, s, dp, ntx, parity, sw);
      break;
    case CP_RESIDENT:
      hipLaunchKernelGGL((step2_kernel<S, CP_RESIDENT, false, SH>), grid, block, 0, s, dp, ntx, parity, sw);
      break;
    default:
      hipLaunchKernelGGL((step2_kernel<S, CP_TUNED, false, SH>), grid, block, 0, s, dp, ntx, parity, sw);
      break;
  }
  return (int)hipGetLastError();
}

int launch_step2(int prec, const void *desc, const void *ddev, int cp, int parity, int sw, int rows, void *stream) {
  switch (prec) {
    case PREC_FP64:
      if (rows != TwoStep<double>::H) return (int)hipErrorInvalidValue;
      return step2_t<double>(desc, ddev, cp, parity, sw, stream);
    case PREC_FP32:
      if (rows != TwoStep<float>::H) return (int)hipErrorInvalidValue;
      return step2_t<float>(desc, ddev, cp, parity, sw, stream);
    default:
      if (rows == TallTwo::H) {
        if (((const Desc<float> *)desc)->nee) return (int)hipErrorInvalidValue;
        return step2_t<_Float16, TallTwo>(desc, ddev, cp, parity, sw, stream);
      }
      if (rows != TwoStep<_Float16>::H) return (int)hipErrorInvalidValue;
      return step2_t<_Float16>(desc, ddev, cp, parity, sw, stream);
  }
}

template <typename S, typename TS>
static int step3_t(const void *desc, const void *ddev, int cp, int parity, int sw, void *stream) {
  const auto &d = *(const Desc<typename St<S>::R> *)desc;
  const auto *dp = (const Desc<typename St<S>::R> *)ddev;
  hipStream_t s = (hipStream_t)stream;
  constexpr int W = TS::W, H = TS::H;
  const int ntx = (d.nx + W - 1) / W, nty = (d.ny + H - 1) / H;
  const dim3 grid(ntx * nty), block(TS::THREADS);
  switch (cp) {
    case CP_STREAM: hipLaunchKernelGGL((step3_kernel<S, CP_STREAM, TS>), grid, block, 0, s, dp, ntx, parity, sw); break;
    case CP_RESIDENT:
      hipLaunchKernelGGL((step3_kernel<S, CP_RESIDENT, TS>), grid, block, 0, s, dp, ntx, parity, sw);
      break;
    default: hipLaunchKernelGGL((step3_kernel<S, CP_TUNED, TS>), grid, block, 0, s, dp, ntx, parity, sw); break;
  }
  return (int)hipGetLastError();
}

int launch_step3(int prec, const void *desc, const void *ddev, int cp, int parity, int sw, int rows, void *stream) {
  const auto nee = [&](auto *dp) { return dp->nee != 0; };
  switch (prec) {
    case PREC_FP64:
      if (nee((const Desc<double> *)desc) || rows != ThreeStep<double>::H) return (int)hipErrorInvalidValue;
      return step3_t<double, ThreeStep<double>>(desc, ddev, cp, parity, sw, stream);
    case PREC_FP32:
      if (nee((const Desc<float> *)desc)) return (int)hipErrorInvalidValue;
      if (rows == TallThree::H) return step3_t<float, TallThree>(desc, ddev, cp, parity, sw, stream);
      if (rows != ThreeStep<float>::H) return (int)hipErrorInvalidValue;
      return step3_t<float, ThreeStep<float>>(desc, ddev, cp, parity, sw, stream);
    default: return (int)hipErrorInvalidValue;   // FP16 storage: one or two steps per launch
  }
}

template <typename S, typename SH>
static void batch2_shape(int cp, const Desc<typename St<S>::R> *dd, const Item *items, const int *range, int grid,
                         int parity, hipStream_t s) {
  const dim3 block(SH::THREADS);
  switch (cp) {
    case CP_STREAM:
      hipLaunchKernelGGL((step2_batch_kernel<S, CP_STREAM, SH>), dim3(grid), block, 0, s, dd, items, range, parity);
      break;
    case CP_RESIDENT:
      hipLaunchKernelGGL((step2_batch_kernel<S, CP_RESIDENT, SH>), dim3(grid), block, 0, s, dd, items, range, parity);
      break;
    default:
      hipLaunchKernelGGL((step2_batch_kernel<S, CP_TUNED, SH>), dim3(grid), block, 0, s, dd, items, range, parity);
      break;
  }
}

template <typename S>
static void batch2_t(int cp, int shape, const void *descs, const Item *items, const int *range, int grid, int parity,
                     hipStream_t s) {
  using D = Desc<typename St<S>::R>;
  const D *dd = (const D *)descs;
  switch (shape) {
    case 1: batch2_shape<S, typename BatchShape<S, 1>::T>(cp, dd, items, range, grid, parity, s); break;
    case 2: batch2_shape<S, typename BatchShape<S, 2>::T>(cp, dd, items, range, grid, parity, s); break;
    default: batch2_shape<S, typename BatchShape<S, 0>::T>(cp, dd, items, range, grid, parity, s); break;
  }
}

int launch_step2_batch(int prec, int cp, int shape, const void *descs, const Item *items, const int *range, int grid,
                       int parity, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (prec) {
    case PREC_FP64: batch2_t<double>(cp, shape, descs, items, range, grid, parity, s); break;
    case PREC_FP32: batch2_t<float>(cp, shape, descs, items, range, grid, parity, s); break;
    default: batch2_t<_Float16>(cp, shape, descs, items, range, grid, parity, s); break;
  }
  return (int)hipGetLastError();
}

template <typename S>
static void batch3_t(int cp, const void *descs, const Item *items, const int *range, int grid, int parity,
                     hipStream_t s) {
  using D = Desc<typename St<S>::R>;
  const D *dd = (const D *)descs;
  const dim3 block(ThreeStep<S>::THREADS);
  switch (cp) {
    case CP_STREAM:
      hipLaunchKernelGGL((step3_batch_kernel<S, CP_STREAM>), dim3(grid), block, 0, s, dd, items, range, parity);
      break;
    case CP_RESIDENT:
      hipLaunchKernelGGL((step3_batch_kernel<S, CP_RESIDENT>), dim3(grid), block, 0, s, dd, items, range, parity);
      break;
    default:
      hipLaunchKernelGGL((step3_batch_kernel<S, CP_TUNED>), dim3(grid), block, 0, s, dd, items, range, parity);
      break;
  }
}

template <typename S>
static void batch2_nee_t(int cp, const void *descs, const Item *items, const int *range, int grid, int parity,
                         hipStream_t s) {
  using D = Desc<typename St<S>::R>;
  const D *dd = (const D *)descs;
  const dim3 block(TwoStep<S>::THREADS);
  switch (cp) {
    case CP_STREAM:
      hipLaunchKernelGGL((step2_batch_nee_kernel<S, CP_STREAM>), dim3(grid), block, 0, s, dd, items, range, parity);
      break;
    case CP_RESIDENT:
      hipLaunchKernelGGL((step2_batch_nee_kernel<S, CP_RESIDENT>), dim3(grid), block, 0, s, dd, items, range, parity);
      break;
    default:
      hipLaunchKernelGGL((step2_batch_nee_kernel<S, CP_TUNED>), dim3(grid), block, 0, s, dd, items, range, parity);
      break;
  }
}

int launch_step2_batch_nee(int prec, int cp, const void *descs, const Item *items, const int *range, int grid,
                           int parity, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  static_assert(TwoStep<float>::W == BatchShape<float, 0>::T::W && TwoStep<float>::H == BatchShape<float, 0>::T::H &&
                    TwoStep<double>::W == BatchShape<double, 0>::T::W &&
                    TwoStep<double>::H == BatchShape<double, 0>::T::H,
                "the batched node-wall launch takes tiles of batch tile shape 0");
  switch (prec) {
    case PREC_FP64: batch2_nee_t<double>(cp, descs, items, range, grid, parity, s); break;
    case PREC_FP32: batch2_nee_t<float>(cp, descs, items, range, grid, parity, s); break;
    default: return (int)hipErrorInvalidValue;   // FP16 storage: node walls take one step per launch
  }
  return (int)hipGetLastError();
}

int launch_step3_batch(int prec, int cp, const void *descs, const Item *items, const int *range, int grid,
                       int parity, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  static_assert(ThreeStep<float>::W == BatchShape<float, 0>::T::W && ThreeStep<float>::H == BatchShape<float, 0>::T::H &&
                    ThreeStep<double>::W == BatchShape<double, 0>::T::W &&
                    ThreeStep<double>::H == BatchShape<double, 0>::T::H,
                "the batched three-step launch takes the items of batch tile shape 0");
  switch (prec) {
    case PREC_FP64: batch3_t<double>(cp, descs, items, range, grid, parity, s); break;
    case PREC_FP32: batch3_t<float>(cp, descs, items, range, grid, parity, s); break;
    default: return (int)hipErrorInvalidValue;   // FP16 storage: one or two steps per launch
  }
  return (int)hipGetLastError();
}

void two_step_tile_shape(int prec, int *w, int *h) {
  *w = prec == PREC_FP64 ? TwoStep<double>::W : TwoStep<float>::W;
  *h = prec == PREC_FP64 ? TwoStep<double>::H : TwoStep<float>::H;
}

template <typename S, int K>
static void shape_of(int *w, int *h) {
  *w = BatchShape<S, K>::T::W;
  *h = BatchShape<S, K>::T::H;
}

int batch_tile_shapes() { return kBatchShapes; }

void batch_tile_shape(int prec, int shape, int *w, int *h) {
  const int k = shape < 0 || shape >= kBatchShapes ? 0 : shape;
  if (prec == PREC_FP64) {
    if (k == 0) shape_of<double, 0>(w, h);
    else if (k == 1) shape_of<double, 1>(w, h);
    else shape_of<double, 2>(w, h);
  } else {
    if (k == 0) shape_of<float, 0>(w, h);
    else if (k == 1) shape_of<float, 1>(w, h);
    else shape_of<float, 2>(w, h);
  }
}

template <typename S>
static void batch_t(int cp, const void *descs, const Item *items, const int *range, int grid, int parity,
                    hipStream_t s) {
  using D = Desc<typename St<S>::R>;
  const D *dd = (const D *)descs;
  switch (cp) {
    case CP_STREAM:
      hipLaunchKernelGGL((step_batch_kernel<S, CP_STREAM>), dim3(grid), dim3(256), 0, s, dd, items, range, parity);
      break;
    case CP_RESIDENT:
      hipLaunchKernelGGL((step_batch_kernel<S, CP_RESIDENT>), dim3(grid), dim3(256), 0, s, dd, items, range, parity);
      break;
    default:
      hipLaunchKernelGGL((step_batch_kernel<S, CP_TUNED>), dim3(grid), dim3(256), 0, s, dd, items, range, parity);
      break;
  }
}

int launch_step_batch(int prec, int cp, const void *descs, const Item *items, const int *range, int grid, int parity,
                      void *stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (prec) {
    case PREC_FP64: batch_t<double>(cp, descs, items, range, grid, parity, s); break;
    case PREC_FP32: batch_t<float>(cp, descs, items, range, grid, parity, s); break;
    default: batch_t<_Float16>(cp, descs, items, range, grid, parity, s); break;
  }
  return (int)hipGetLastError();
}

int observables_blocks(int ny) { return (ny + OBS_ROWS - 1) / OBS_ROWS; }

template <typename S>
static int obs_t(const void *desc, int parity, void *snap, double *partials, int nblocks, double *out,
                 const double *wT, const double *wC, double LdT, double LdC, void *stream) {
  using R = typename St<S>::R;
  const auto &d = *(const Desc<R> *)desc;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(obs_partial_kernel<S>, dim3(nblocks), dim3(OBS_THREADS), 0, s, d, parity, (R *)snap,
                     partials);
  hipLaunchKernelGGL(obs_final_kernel, dim3(NSLOT), dim3(OBS_THREADS), 0, s, partials, nblocks, out);
  hipLaunchKernelGGL(wall_kernel<R>, dim3(4), dim3(256), 0, s, d, wT, wC, LdT, LdC, out);
  return (int)hipGetLastError();
}

int launch_observables(int prec, const void *desc, int parity, void *snap, double *partials, int nblocks,
                       double *out, const double *wT, const double *wC, double LdT, double LdC,
                       void *stream) {
  switch (prec) {
    case PREC_FP64: return obs_t<double>(desc, parity, snap, partials, nblocks, out, wT, wC, LdT, LdC, stream);
    case PREC_FP32: return obs_t<float>(desc, parity, snap, partials, nblocks, out, wT, wC, LdT, LdC, stream);
    default: return obs_t<_Float16>(desc, parity, snap, partials, nblocks, out, wT, wC, LdT, LdC, stream);
  }
}

// ---------------------------------------------------------------- fixed scratch
// Device memory of lbm_observables_static, for callers that cannot allocate: the result slots,
// the per-block partial sums of the observables of a lattice of up to kStaticRows rows, and the
// staging of the exported FP64 fields of a lattice of up to kStaticNodes nodes.  One copy per
// device, held until the process ends, shared by every context on that device.
constexpr int kStaticRows = 16384;
constexpr long long kStaticNodes = 1LL << 20;
constexpr long long kStaticOut = 32;
constexpr long long kStaticPartials = (long long)((kStaticRows + OBS_ROWS - 1) / OBS_ROWS) * NSLOT;
constexpr long long kStaticDoubles = kStaticOut + kStaticPartials + 5 * kStaticNodes;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticDoubles];

StaticScratchLayout static_scratch_layout() {
  StaticScratchLayout l;
  l.max_rows = kStaticRows;
  l.max_nodes = kStaticNodes;
  l.out = 0;
  l.partials = kStaticOut;
  l.fields = kStaticOut + kStaticPartials;
  l.doubles = kStaticDoubles;
  return l;
}

// The address of `scratch` on `device`, which must be the current device: looked up with
// hipGetSymbolAddress on the first call for that device and kept per device (each device holds
// its own copy of the array at its own address).  In host code the name `scratch` is only a
// stand-in: the address returned here is the one kernels and copies must use.
int static_scratch_address(int device, double **ptr) {
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    addr[device] = (double *)p;
  }
  *ptr = addr[device];
  return (int)hipSuccess;
}

template <typename S>
static int export_t(const void *desc, int parity, double *fields, void *stream) {
  const auto &d = *(const Desc<typename St<S>::R> *)desc;
  dim3 grid((d.nx + 255) / 256, d.ny);
  hipLaunchKernelGGL(export_kernel<S>, grid, dim3(256), 0, (hipStream_t)stream, d, parity, fields);
  return (int)hipGetLastError();
}

int launch_export(int prec, const void *desc, int parity, double *fields, void *stream) {
  switch (prec) {
    case PREC_FP64: return export_t<double>(desc, parity, fields, stream);
    case PREC_FP32: return export_t<float>(desc, parity, fields, stream);
    default: return export_t<_Float16>(desc, parity, fields, stream);
  }
}

}  // namespace lbmk
