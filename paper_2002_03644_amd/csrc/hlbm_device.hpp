// Device code of the D2Q9 hybrid LBM step for gfx950 (MI355X).
//
// Included by the per-precision translation units (hlbm_kernels_f32.hip,
// hlbm_kernels_f64.hip) with HLBM_REAL defined.  The arithmetic follows the
// HLBM of arXiv 2002.03644 in moment (Hermite-coefficient) space:
//   - moments rho, rho u, Pi from the populations (Eqs. rhoalgo, ualgo);
//   - theta from the entropy closure (Eq. Entropie expression), p = rho c_s^2
//     theta (Eq. perfect gas), local tau = mu / p, taubar = tau + 1/2 (Sec. 3.1);
//   - lattice-closure correction E1 = d_a(rho u_a (1 - theta - u_a^2)) by the
//     upwind difference of Sec. 3.2 (sgn(u) = 0, i.e. centred, for |u| within
//     the rounding band sgn_eps), E2 = p (2 - gamma) div u (Eq. E2 corr term);
//   - HRR stress a1 = sigma a1PR + (1 - sigma) a1FD (Eq. a1sigalgo), with a1PR in
//     closed form (the projection of F - f^eq + psi/2 on H_ab) and a1FD from
//     centred velocity gradients (Eq. a1FD), and the recursion to xxy, yyx,
//     xxyy (Sec. 3.3);
//   - post-collision populations f* = f^eq + (1 - 1/taubar) f^1 + psi/2
//     (Eq. streamalgo) as one projection of nine Hermite coefficients;
//   - pull streaming F'_i(x) = f*_i(x - c_i);
//   - entropy update (Eq. sequaalgo): upwind MUSCL with the van Albada slope,
//     5-point Fourier term, viscous heat Phi (Eq. viscous heat discret or the
//     finite-difference form), explicit Euler.
//
// Data layout in HBM: ten planes [p][ny][nx] (x fastest), p = 0..8 the
// populations and p = 9 the entropy; two such buffers are ping-ponged.  In
// the FP32 form the planes hold deviations g_i = F_i - f^eq_i(rho_ref, 0,
// theta_ref) and ds = s - s_ref, which keeps the small fluctuations that
// drive the dynamics out of the rounding of the O(1) rest state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#if !defined(HLBM_REAL) || !defined(HLBM_NS)
#error "define HLBM_REAL and HLBM_NS before including hlbm_device.hpp"
#endif

namespace hlbm {
namespace HLBM_NS {  // one namespace per precision: no shared symbols

using real = HLBM_REAL;

constexpr int kQ = 9;
constexpr int kPlanes = 10;

// Arguments shared by every per-domain kernel.
struct DomainArgs {
  long long plane;     // elements per plane (padded)
  int nx, ny, bcx, bcy;
  int pitch;           // elements per state row (nx rounded up to 64)
  int flags;           // bit 0: Phi by finite differences, bit 1: centred E1, bit 2: no E2,
                       // bit 3: precise theta, bit 4: third-order expansion
  real mu, sigma, lambda, inv_cv, gm1, e2c, gamma, sgn_eps;
  real rho_ref, theta_ref, log_rho_ref, s_ref;
  real fref[kQ];       // deviation reference populations (zero in the FP64 form)
  real wall_u_lo, wall_u_hi, wall_theta;  // bcy == kBcWall: wall velocities, temperature
};

// State offset (within a plane) of node i = y nx + x of the dense [ny][nx]
// order used by the field arrays.
__device__ __forceinline__ long long state_off(const DomainArgs &d, long long i) {
  if (d.pitch == d.nx) return i;
  const int y = (int)(i / d.nx);
  return (long long)y * d.pitch + (i - (long long)y * d.nx);
}

struct StepArgs {
  DomainArgs d;
  const real *src;     // plane 0 of the state read this step
  real *dst;           // plane 0 of the state written
  unsigned *status;    // bit 0 set when a node diverged
  int rows;            // output rows per strip
  int nbx, nby;        // workgroups along x and y
  int xcd_remap;       // 1: spread spatial neighbours onto the same XCD
};

constexpr int kFlagPhiFD = 1, kFlagE1Centred = 2, kFlagE2Off = 4;
constexpr int kFlagPreciseTheta = 8;  // theta - theta_ref from expm1 / log1p (see node_dtheta)
// Hermite expansion truncated at third order (the original model of Sec. 2.3):
// the xxyy coefficient of every projected population, equilibrium and
// off-equilibrium alike, is zero (the deviation reference drops it too).
constexpr int kFlagFeq3 = 16;
constexpr int kBcWall = 2;  // rows y = 0 and y = ny - 1 are walls (ghosts beyond them clamp)

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int map_index(int v, int n, int bc) {
  if (bc == 0) {
    int r = v % n;
    return r < 0 ? r + n : r;
  }
  return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_fast(double x) { return 1.0 / x; }
__device__ __forceinline__ float div_fast(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double div_fast(double a, double b) { return a / b; }
__device__ __forceinline__ float exp_r(float x) { return __expf(x); }
__device__ __forceinline__ double exp_r(double x) { return exp(x); }
__device__ __forceinline__ float log_r(float x) { return __logf(x); }
__device__ __forceinline__ double log_r(double x) { return log(x); }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }

constexpr double kCs2 = 1.0 / 3.0;

// Global access through a uniform base pointer and a 32-bit byte offset, so
// the address is SGPR base + VGPR offset (no 64-bit address arithmetic).
__device__ __forceinline__ real load_at(const real *base, unsigned byte_off) {
  return *(const real *)((const char *)base + byte_off);
}
__device__ __forceinline__ void store_at(real *base, unsigned byte_off, real v) {
  *(real *)((char *)base + byte_off) = v;
}
// Streaming store: the new state is not read again before the whole grid is
// written, so it bypasses cache retention.
__device__ __forceinline__ void store_stream(real *base, unsigned byte_off, real v) {
  __builtin_nontemporal_store(v, (real *)((char *)base + byte_off));
}

// Projection of the nine Hermite coefficients onto the D2Q9 populations:
// f_i = w_i [A0 + c.A/cs2 + H2:A2/(2 cs2^2) + (Hxxy Axxy + Hyyx Ayyx)/(2 cs2^3)
//            + Hxxyy Axxyy/(4 cs2^4)], written out per velocity class.
__device__ __forceinline__ void project(real A0, real Ax, real Ay, real Axx, real Axy, real Ayy,
                                        real Axxy, real Axyy, real Axxyy, real f[kQ]) {
  const real b0 = A0 - real(1.5) * (Axx + Ayy) + real(2.25) * Axxyy;
  f[0] = real(4.0 / 9.0) * b0;
  const real bx = A0 + real(3) * Axx - real(1.5) * Ayy - real(4.5) * Axxyy;
  const real ox = real(3) * Ax - real(4.5) * Axyy;
  f[1] = real(1.0 / 9.0) * (bx + ox);
  f[3] = real(1.0 / 9.0) * (bx - ox);
  const real by = A0 + real(3) * Ayy - real(1.5) * Axx - real(4.5) * Axxyy;
  const real oy = real(3) * Ay - real(4.5) * Axxy;
  f[2] = real(1.0 / 9.0) * (by + oy);
  f[4] = real(1.0 / 9.0) * (by - oy);
  const real bd = A0 + real(3) * (Axx + Ayy) + real(9) * Axxyy;
  const real dxy = real(9) * Axy;
  const real dx = real(3) * Ax + real(9) * Axyy;
  const real dy = real(3) * Ay + real(9) * Axxy;
  f[5] = real(1.0 / 36.0) * ((bd + dxy) + (dx + dy));
  f[6] = real(1.0 / 36.0) * ((bd - dxy) - (dx - dy));
  f[7] = real(1.0 / 36.0) * ((bd + dxy) - (dx + dy));
  f[8] = real(1.0 / 36.0) * ((bd - dxy) + (dx - dy));
}

// Node moments from the stored planes.  dr = rho - rho_ref (rho itself in the
// FP64 form), Pi deviations likewise relative to the rest state p_ref I.
struct NodeMoments {
  real dr, rho, jx, jy, pxx, pyy, pxy;
};

__device__ __forceinline__ NodeMoments node_moments(const real F[kQ], const DomainArgs &d) {
  NodeMoments m;
  real r = ((F[0] + F[1]) + (F[2] + F[3])) + ((F[4] + F[5]) + (F[6] + F[7])) + F[8];
  m.dr = r;
  m.rho = r + d.rho_ref;
  m.jx = ((F[1] - F[3]) + (F[5] - F[7])) + (F[8] - F[6]);
  m.jy = ((F[2] - F[4]) + (F[5] - F[7])) + (F[6] - F[8]);
  const real diag = (F[5] + F[6]) + (F[7] + F[8]);
  m.pxx = (F[1] + F[3]) + diag;
  m.pyy = (F[2] + F[4]) + diag;
  m.pxy = (F[5] - F[6]) + (F[7] - F[8]);
  return m;
}

// theta from the stored entropy (deviation form: ds = s - s_ref).
__device__ __forceinline__ real node_theta(real rho, real sv, const DomainArgs &d) {
  return d.theta_ref * exp_r(sv * d.inv_cv + d.gm1 * (log_r(rho) - d.log_rho_ref));
}

// theta - theta_ref with relative accuracy on the deviation itself:
// theta_ref expm1(ds / c_v + (gamma - 1) ln(rho / rho_ref)), the density ratio
// from dr = rho - rho_ref in FP32 (log1p), rho itself in the FP64 form
// (rho_ref = 0, theta_ref = 1 there).  The Fourier term's Laplacian is taken
// of these deviations: in slow, well-resolved flows the temperature
// differences between neighbours are a few 1e-6 of theta, which absolute
// FP32 values would round to a few per cent.
//
// FP32 uses the hardware exp and log with the classic corrections that make
// them accurate relative to small results: Goldberg's log1p(y) = ln(u) y /
// (u - 1) with u = 1 + y, exact when u rounds to 1, and expm1 by its Taylor
// series for |x| < 1/4, else Kahan's (u - 1) x / ln(u) with u = e^x.  FP64
// uses the library functions.
__device__ __forceinline__ float log1p_fast(float y) {
  const float u = 1.0f + y;
  const float um1 = u - 1.0f;
  return um1 == 0.0f ? y : __logf(u) * div_fast(y, um1);
}
__device__ __forceinline__ float expm1_fast(float x) {
  // |x| < 1/4: the Taylor series to x^7 (truncation below 1e-9 of the result)
  if (fabsf(x) < 0.25f) {
    const float p = 1.0f / 5040.0f;
    return x * (1.0f + x * (0.5f + x * (1.0f / 6.0f + x * (1.0f / 24.0f +
                x * (1.0f / 120.0f + x * (1.0f / 720.0f + x * p))))));
  }
  const float u = __expf(x);
  const float um1 = u - 1.0f;
  if (um1 == -1.0f) return -1.0f;
  return um1 * div_fast(x, __logf(u));
}
__device__ __forceinline__ float node_dtheta(float dr, float rho, float sv, const DomainArgs &d) {
  return d.theta_ref * expm1_fast(sv * d.inv_cv + d.gm1 * log1p_fast(dr / d.rho_ref));
}
__device__ __forceinline__ double node_dtheta(double dr, double rho, double sv,
                                              const DomainArgs &d) {
  return d.theta_ref * expm1(sv * d.inv_cv + d.gm1 * (log(rho) - d.log_rho_ref));
}

// van Albada limited slope b phi(a/b), phi(r) = (r^2 + r)/(r^2 + 1), zero for
// a b <= 0; written as a b (a + b)/(a^2 + b^2).  Differences so small that
// a^2 + b^2 leaves the normal range (below 1e-30 in FP32, where the stored
// entropy deviation can reach them) give the limit value 0 instead of 0/0.
__device__ __forceinline__ real tiny_sq() { return sizeof(real) == 4 ? real(1e-30) : real(1e-300); }
__device__ __forceinline__ real van_albada(real a, real b) {
  const real ab = a * b;
  const real den = a * a + b * b;
  return (ab > real(0) && den > tiny_sq()) ? div_fast(ab * (a + b), den) : real(0);
}

// Upwind MUSCL derivative scaled by |u|: for u > 0 the stencil (q_{-1}, q0,
// q1, q2) = (s_{i+1}, s_i, s_{i-1}, s_{i-2}); for u < 0 the mirror image.
// Both signs reduce to |u| [(q0 - q1) + (slope(q0) - slope(q1)) / 2] by the
// odd symmetry of the limiter.  u = 0 gives 0.
__device__ __forceinline__ real muscl_term(real u, real sm2, real sm1, real s0, real sp1,
                                           real sp2) {
  const bool pos = u > real(0);
  const real qm1 = pos ? sp1 : sm1;
  const real q1 = pos ? sm1 : sp1;
  const real q2 = pos ? sm2 : sp2;
  const real d01 = s0 - q1;
  const real sl0 = van_albada(d01, qm1 - s0);
  const real sl1 = van_albada(q1 - q2, d01);
  return __builtin_fabs(u) * (d01 + real(0.5) * (sl0 - sl1));
}

// --------------------------------------------------------------- the step
//
// One workgroup owns a tile of CW output columns (x0 a multiple of CW, so
// every row segment it stores is aligned) and `rows` output rows, plus a
// radius-2 halo.  Lanes 0..CW-1 handle the tile's columns; an extra wave
// holds the four halo columns (x0-2, x0-1, x0+CW, x0+CW+1) on its first four
// lanes.  In the LDS rings a column sits at position ri = column - (x0 - 2).
// Each lane sweeps the rows of the strip through three stages:
//   A(j)    moments of row j from the ten planes: u, theta, Gamma and s go
//           into LDS rings, rho and Pi stay in registers;
//   B(k)    gradients, E, a1 and the nine post-collision populations of row
//           k (radius-1 stencil through the rings): the six with c_x != 0
//           into LDS rings, the three with c_x = 0 into the lane's registers;
//   C(k)    pull streaming of row k out of those and its entropy update
//           (radius-2 stencil), storing both.
// Iteration i issues the loads of row i+1, runs B(i-1), a barrier, A(i+1) on
// those loads, C(i-2), and a second barrier.  Loads are thus consumed in the
// iteration that issued them, after the B work that hides their latency, and
// before C's stores (a wait placed after stores that sit under a branch
// would also wait for the stores).  Each node's moments and collision are
// computed once per step (plus a 4-column halo); HBM sees one read and one
// write of the state.
//
// Ring depths are the smallest the two barriers per iteration allow (only a
// write of A(i+1) may overlap a read of C(i-2) of another wave):
//   u_x, u_y, Gamma_x: 2 rows (B reads the x-neighbours of row k; rows k-1
//   and k+1 of its own column, and Gamma_y entirely, come from registers);
//   theta: 5 (C reads rows k-1 and k+1);  s: 6 (C reads rows k-2..k+2);
//   post-collision populations by the row they stream from: c_y = 0 -> 2,
//   c_y = +1 (read one row later) -> 3, c_y = -1 (read in the same row) -> 1;
//   in registers the same delays: population 0 one row, 2 two rows, 4 none.
// 29 rows of CW + 4 floats in all: 22.7 KB at CW = 192, seven workgroups per
// CU.
// Shared memory of one tile sweep.
template <int CW>
struct TileRings {
  static constexpr int W = CW + 4;  // ring width: tile plus halo
  real ux[2][W], uy[2][W], gx[2][W];
  real th[5][W], s[6][W];
  // post-collision populations that stream across columns; 0, 2 and 4
  // (c_x = 0) stay in their lane's registers
  real f0[2][2][W];  // populations 1, 3   (c_y =  0)
  real fp[3][2][W];  // populations 5, 6   (c_y = +1)
  real fm[2][W];     // populations 7, 8   (c_y = -1)
};

// Batched items: the skip of a frozen domain is decided once per item for
// the whole workgroup (another workgroup can set the flag at any moment, and
// waves that read it at different times would disagree and pair up barriers
// across items).  Every thread reads the flag word before the item's first
// loads are issued (one request per wave, no branch, so no wait for it is
// placed before those loads); the sweep's first barrier, an OR over the
// threads, then decides for all of them, so the flag's latency overlaps the
// loads.
__device__ __forceinline__ unsigned domain_frozen(const unsigned *status) {
  return __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool kBatch>
__device__ __forceinline__ bool barrier_skip(unsigned frozen) {
  if constexpr (kBatch) return __syncthreads_or(frozen != 0u) != 0;
  __syncthreads();
  return false;
}

// One tile (bx, by) of one domain: src / dst point at plane 0 of the two
// state buffers, planes are `d.plane` elements apart.  Ends with a barrier,
// so the rings can be reused by the next tile.  kBatch: returns after the
// prologue when any thread's `frozen` is nonzero (see domain_frozen).
template <int CW, bool kBatch = false>
__device__ __forceinline__ void sweep_tile(const DomainArgs &d, const real *src0, real *dst0,
                                           unsigned *status, const int rows, const int bx,
                                           const int by, const unsigned frozen, TileRings<CW> &R) {
  const int t = threadIdx.x;
  const real *src[kPlanes];
  real *dst[kPlanes];
#pragma unroll
  for (int q = 0; q < kPlanes; ++q) {
    src[q] = src0 + (long long)q * d.plane;
    dst[q] = dst0 + (long long)q * d.plane;
  }
  auto &r_ux = R.ux;
  auto &r_uy = R.uy;
  auto &r_gx = R.gx;
  auto &r_th = R.th;
  auto &r_s = R.s;
  auto &r_f0 = R.f0;
  auto &r_fp = R.fp;
  auto &r_fm = R.fm;
  const int x0 = bx * CW, y0 = by * rows;
  // lane -> ring position: tile lanes at 2..CW+1, halo lanes at 0, 1, CW+2, CW+3
  const int h = t - CW;
  const int ri = t < CW ? t + 2 : (h < 2 ? h : (h < 4 ? CW + h : 0));
  const bool a_lane = t < CW + 4;                        // loads and moments
  const bool b_col = t < CW || h == 1 || h == 2;         // collision: ring 1..CW+2
  const int vx = x0 - 2 + ri;
  const int cx = map_index(vx, d.nx, d.bcx);
  const int nrow = min(rows, d.ny - y0);
  const int nit = nrow + 4;
  const bool own_col = t < CW && vx < d.nx;
  const real cs2 = real(kCs2);
  const real cref = cs2 * (d.theta_ref - real(1));
  constexpr unsigned kEl = sizeof(real);
  unsigned bad = 0;

  // 32-bit byte offset of virtual row j (x fastest) from the plane bases.
  auto row_off = [&](int j) {
    return (unsigned)(map_index(y0 - 2 + j, d.ny, d.bcy) * d.pitch + cx) * kEl;
  };

  // Node state of rows k (s0_*) and k+1 (s1_*) carried from A to B.
  real s0_dr = 0, s0_rho = 1, s0_pxx = 0, s0_pyy = 0, s0_pxy = 0, s0_ux = 0, s0_uy = 0, s0_th = 1;
  real s1_dr = 0, s1_rho = 1, s1_pxx = 0, s1_pyy = 0, s1_pxy = 0, s1_ux = 0, s1_uy = 0, s1_th = 1;
  // B's stencil along y within the lane's own column, in registers: u of row
  // k-1 and Gamma_y = rho u_y (1 - theta - u_y^2) of rows k-1, k, k+1
  real m_ux = 0, m_uy = 0, m_gy = 0, c_gy = 0, n_gy = 0;
  // B -> C carry: B(k) fills nB_*, copied to cB_* at the end of the
  // iteration, read by C(k) in the next one.
  real nB_ux = 0, nB_uy = 0, nB_rho = 1, nB_th = 1, nB_phi = 0;
  real cB_ux = 0, cB_uy = 0, cB_rho = 1, cB_th = 1, cB_phi = 0;
  // populations 0, 2, 4 of B's rows kept in registers: nB_* of row k (this
  // iteration's B), cB_f0 of row k-1, cB_f2 of row k-1, cB_f2b of row k-2
  real nB_f0 = 0, nB_f2 = 0, nB_f4 = 0, cB_f0 = 0, cB_f2 = 0, cB_f2b = 0;

  // A(j): moments of one row from its ten loaded planes.
  auto stage_a = [&](const int j, const real (&ld)[kPlanes]) {
    real F[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) F[q] = ld[q];
    const real sv = ld[9];
    const NodeMoments m = node_moments(F, d);
    const real inv_rho = rcp_fast(m.rho);
    const real ux = m.jx * inv_rho, uy = m.jy * inv_rho;
    // The Fourier term's Laplacian is taken of what the theta ring holds:
    // theta itself by default, theta - theta_ref (accurate relative to
    // itself) with the precise-theta flag; the constant shift cancels.
    real th, lap_val;
    if (d.flags & kFlagPreciseTheta) {
      lap_val = node_dtheta(m.dr, m.rho, sv, d);
      th = d.theta_ref + lap_val;
    } else {
      th = node_theta(m.rho, sv, d);
      lap_val = th;
    }
    r_ux[j & 1][ri] = ux;
    r_uy[j & 1][ri] = uy;
    r_th[j % 5][ri] = lap_val;
    r_gx[j & 1][ri] = m.rho * ux * ((real(1) - th) - ux * ux);
    r_s[j % 6][ri] = sv;
    m_ux = s0_ux;
    m_uy = s0_uy;
    m_gy = c_gy;
    c_gy = n_gy;
    n_gy = m.rho * uy * ((real(1) - th) - uy * uy);
    s0_dr = s1_dr;
    s0_rho = s1_rho;
    s0_pxx = s1_pxx;
    s0_pyy = s1_pyy;
    s0_pxy = s1_pxy;
    s0_ux = s1_ux;
    s0_uy = s1_uy;
    s0_th = s1_th;
    s1_dr = m.dr;
    s1_rho = m.rho;
    s1_pxx = m.pxx;
    s1_pyy = m.pyy;
    s1_pxy = m.pxy;
    s1_ux = ux;
    s1_uy = uy;
    s1_th = th;
    bad |= (m.rho > real(0) && th > real(0) && __builtin_isfinite(ux + uy + th)) ? 0u : 1u;
  };

  if (a_lane) {  // prologue: A(0)
    real ld[kPlanes];
    const unsigned off = row_off(0);
#pragma unroll
    for (int q = 0; q < kPlanes; ++q) ld[q] = load_at(src[q], off);
    stage_a(0, ld);
  }
  if (barrier_skip<kBatch>(frozen)) return;

  for (int i = 0; i < nit; ++i) {
    // ---------------- issue the loads of row i+1 (consumed by A after B)
    real ld[kPlanes];
    const bool do_a = a_lane && i + 1 < nit;
    if (do_a) {
      const unsigned off = row_off(i + 1);
#pragma unroll
      for (int q = 0; q < kPlanes; ++q) ld[q] = load_at(src[q], off);
    }
    // A(i) has run for rows 0..i; s1_* holds row i, s0_* row i-1.

    // ---------------- B(k), k = i-1: collision
    if (i >= 2) {
      const int k = i - 1;
      const int sc = k % 3;
      if (b_col) {
        const real rho = s0_rho, ux = s0_ux, uy = s0_uy, th = s0_th;
        const int su = k & 1;
        const real uxe = r_ux[su][ri + 1], uxw = r_ux[su][ri - 1];
        const real uye = r_uy[su][ri + 1], uyw = r_uy[su][ri - 1];
        const real uxn = s1_ux, uxs = m_ux;
        const real uyn = s1_uy, uys = m_uy;
        const real dxux = real(0.5) * (uxe - uxw), dxuy = real(0.5) * (uye - uyw);
        const real dyux = real(0.5) * (uxn - uxs), dyuy = real(0.5) * (uyn - uys);
        const real div = dxux + dyuy;
        const real p = rho * cs2 * th;
        const real dth = th - d.theta_ref;
        const real dp = cs2 * (s0_dr * th + d.rho_ref * dth);  // p - p_ref
        const real tau = div_fast(d.mu, p);
        const real taub = tau + real(0.5);
        const real itaub = rcp_fast(taub);
        // E1 (upwind in the sign of the node velocity; centred inside the band)
        const real gc = r_gx[k & 1][ri];
        const real gxe = r_gx[k & 1][ri + 1], gxw = r_gx[k & 1][ri - 1];
        const real gcy = c_gy;
        const real gyn = n_gy, gys = m_gy;
        real e1x, e1y;
        if (d.flags & kFlagE1Centred) {
          e1x = real(0.5) * (gxe - gxw);
          e1y = real(0.5) * (gyn - gys);
        } else {
          const real ep = d.sgn_eps;
          e1x = ux > ep ? gc - gxw : (ux < -ep ? gxe - gc : real(0.5) * (gxe - gxw));
          e1y = uy > ep ? gcy - gys : (uy < -ep ? gyn - gcy : real(0.5) * (gyn - gys));
        }
        const real e2 = (d.flags & kFlagE2Off) ? real(0) : d.e2c * p * div;
        const real Exx = e1x + e2, Eyy = e1y + e2;
        // HRR stress
        const real rux = rho * ux, ruy = rho * uy;
        const real ruxx = rux * ux, ruyy = ruy * uy, ruxy = rux * uy;
        const real prxx = (s0_pxx - dp) - ruxx + real(0.5) * Exx;
        const real pryy = (s0_pyy - dp) - ruyy + real(0.5) * Eyy;
        const real prxy = s0_pxy - ruxy;
        const real tp = taub * p;
        const real fdxx = -tp * (dxux - dyuy);
        const real fdxy = -tp * (dyux + dxuy);
        // wall rows take the projected stress alone: their rebuilt populations
        // carry the wall's finite-difference stress
        const int yk = y0 - 2 + k;
        const bool wall_row = d.bcy == kBcWall && (yk == 0 || yk == d.ny - 1);
        const real sg = wall_row ? real(1) : d.sigma, sg1 = real(1) - sg;
        const real a1xx = sg * prxx + sg1 * fdxx;
        const real a1yy = sg * pryy - sg1 * fdxx;
        const real a1xy = sg * prxy + sg1 * fdxy;
        const real c = cs2 * (th - real(1));
        const real a1xxy = uy * a1xx + real(2) * ux * a1xy;
        const real a1xyy = ux * a1yy + real(2) * uy * a1xy;
        const real a1xxyy = real(2) * (ux * a1xyy + uy * a1xxy) + (c - ux * ux) * a1yy +
                            (c - uy * uy) * a1xx - real(4) * ux * uy * a1xy;
        const real om = real(1) - itaub;
        // rho c - rho_ref c_ref and rho c^2 - rho_ref c_ref^2 as deviations
        const real drc = dp - cs2 * s0_dr;
        const real dc = cs2 * dth;
        const real drc2 = s0_dr * c * c + d.rho_ref * dc * (c + cref);
        const real Axx = ruxx + drc + om * a1xx + real(0.5) * Exx;
        const real Ayy = ruyy + drc + om * a1yy + real(0.5) * Eyy;
        const real Axy = ruxy + om * a1xy;
        const real rc = rho * c;
        const real Axxy = ruxx * uy + rc * uy + om * a1xxy;
        const real Axyy = ruyy * ux + rc * ux + om * a1xyy;
        const real Axxyy = (d.flags & kFlagFeq3)
                               ? real(0)
                               : ruxx * uy * uy + rc * (ux * ux + uy * uy) + drc2 + om * a1xxyy;
        real f[kQ];
        project(s0_dr, rux, ruy, Axx, Axy, Ayy, Axxy, Axyy, Axxyy, f);
        r_f0[k & 1][0][ri] = f[1];
        r_f0[k & 1][1][ri] = f[3];
        r_fp[sc][0][ri] = f[5];
        r_fp[sc][1][ri] = f[6];
        r_fm[0][ri] = f[7];
        r_fm[1][ri] = f[8];
        nB_f0 = f[0];
        nB_f2 = f[2];
        nB_f4 = f[4];
        real phi;
        if (d.flags & kFlagPhiFD) {
          const real aa = dxux - dyuy, bb = dyux + dxuy;
          phi = d.mu * (aa * aa + bb * bb);
        } else {
          phi = -(tau * itaub) * (a1xx * dxux + a1xy * (dyux + dxuy) + a1yy * dyuy);
        }
        nB_ux = ux;
        nB_uy = uy;
        nB_rho = rho;
        nB_th = th;
        nB_phi = phi;
      }
    }
    __syncthreads();

    // ---------------- A(i+1) on the loads issued at the top.  It runs before
    // C so that waiting for those loads never waits for C's stores as well
    // (A writes ring slots of row i+1, which C does not read).
    if (do_a) stage_a(i + 1, ld);

    // ---------------- C(k), k = i-2: stream and entropy
    if (i >= 4 && own_col) {
      const int k = i - 2;
      const int z = k & 1, pm = (k + 2) % 3;  // slot of row k in r_f0, of row k-1 in r_fp
      real Fo[kQ];
      Fo[0] = cB_f0;    // row k, this column
      Fo[1] = r_f0[z][0][ri - 1];
      Fo[3] = r_f0[z][1][ri + 1];
      Fo[2] = cB_f2b;   // row k-1, this column
      Fo[5] = r_fp[pm][0][ri - 1];
      Fo[6] = r_fp[pm][1][ri + 1];
      Fo[4] = nB_f4;    // row k+1, this column
      Fo[7] = r_fm[0][ri + 1];
      Fo[8] = r_fm[1][ri - 1];
      const int s0 = k % 6, s1 = (k + 1) % 6, s2 = (k + 2) % 6, sm1 = (k + 5) % 6,
                sm2 = (k + 4) % 6;
      const real sc = r_s[s0][ri];
      const real advx = muscl_term(cB_ux, r_s[s0][ri - 2], r_s[s0][ri - 1], sc, r_s[s0][ri + 1],
                                   r_s[s0][ri + 2]);
      const real advy = muscl_term(cB_uy, r_s[sm2][ri], r_s[sm1][ri], sc, r_s[s1][ri], r_s[s2][ri]);
      const int t0 = k % 5, tn = (k + 1) % 5, ts = (k + 4) % 5;
      // Laplacian of theta (or of theta - theta_ref, the same)
      const real lap = ((r_th[t0][ri + 1] + r_th[t0][ri - 1]) + (r_th[tn][ri] + r_th[ts][ri])) -
                       real(4) * r_th[t0][ri];
      const real snew = sc - (advx + advy) + div_fast(d.lambda * lap + cB_phi, cB_rho * cB_th);
      const unsigned off = (unsigned)((y0 + k - 2) * d.pitch + vx) * kEl;
#pragma unroll
      for (int q = 0; q < kQ; ++q) store_stream(dst[q], off, Fo[q]);
      store_stream(dst[9], off, snew);
    }
    cB_ux = nB_ux;
    cB_uy = nB_uy;
    cB_rho = nB_rho;
    cB_th = nB_th;
    cB_phi = nB_phi;
    cB_f2b = cB_f2;
    cB_f2 = nB_f2;
    cB_f0 = nB_f0;
    __syncthreads();
  }
  if (bad) atomicOr(status, 1u);
}

// Whole-domain step: one workgroup per tile.
template <int CW>
__global__ __launch_bounds__(CW + 64) void k_step(StepArgs a) {
  __shared__ TileRings<CW> R;
  int bid = blockIdx.x;
  const int nblk = a.nbx * a.nby;
  if (a.xcd_remap) {
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of tiles so halo re-reads stay in its L2.
    const int per = (nblk + 7) >> 3;
    const int xcd = bid & 7, k = bid >> 3;
    const int full = nblk - (per - 1) * 8;  // XCDs that get `per` tiles
    bid = xcd < full ? xcd * per + k : full * per + (xcd - full) * (per - 1) + k;
  }
  sweep_tile<CW>(a.d, a.src, a.dst, a.status, a.rows, bid % a.nbx, bid / a.nbx, 0, R);
}

// Batched step: a persistent grid walks a list of (domain, tile) items in a
// static order (tile_walk; no atomics: the launch can be captured and
// replayed).  Items of a domain whose divergence flag is set are skipped, so
// a diverged domain freezes while the others go on (see domain_frozen).
struct BatchArgs {
  const DomainArgs *doms;
  const long long *offs;  // element offset of each domain's state in a buffer
  const int4 *items;      // (domain, bx, by, strip rows; the kernels read the first three)
  int nitems;
  const real *src_buf;
  real *dst_buf;
  unsigned *status;       // one word per domain
  int rows;
  // tile kernels: when set, the moments (rho, u_x, u_y, theta) of the new
  // state go to mom[c * mom_sc + foffs[domain] + y nx + x], c = 0..3, as
  // k_batch_moments computes them
  real *mom;
  const long long *foffs;
  long long mom_sc;
  // tile kernels: when set, a pending learned correction (moments cx,
  // increments cdl, channel stride mom_sc, per-domain partial sums cparts;
  // see k_corr_apply) is applied to the state as it is loaded, as
  // k_corr_apply would have stored it
  const float *cx, *cdl;
  const double *cparts;
  int cconserve;
  int xcd_walk;  // 1: each XCD walks a contiguous range of the items (see tile_walk)
};

// This workgroup's share of the persistent walk over n items: items first,
// first + step, ... below end.  Workgroups are dealt round-robin to the
// eight XCDs (workgroup b to XCD b mod 8).  With xcd set (and at least eight
// workgroups) the walk gives XCD x the contiguous item range
// [x n / 8, (x + 1) n / 8), taken in order by its workgroups, so tiles and
// strips that share halo rows and columns are loaded through one L2;
// otherwise workgroup b takes every gridDim.x-th item from b.
struct TileWalk {
  int first, step, end;
};
__device__ __forceinline__ TileWalk tile_walk(const int n, const int xcd) {
  const int g = (int)gridDim.x, b = (int)blockIdx.x;
  if (!xcd || g < 8) return TileWalk{b, g, n};
  const int x = b & 7;
  const int lo = (int)((long long)x * n / 8), hi = (int)((long long)(x + 1) * n / 8);
  return TileWalk{lo + (b >> 3), (g - x + 7) >> 3, hi};
}

template <int CW>
__global__ __launch_bounds__(CW + 64) void k_step_batch(BatchArgs a) {
  __shared__ TileRings<CW> R;
  const TileWalk walk = tile_walk(a.nitems, a.xcd_walk);
  for (int it = walk.first; it < walk.end; it += walk.step) {
    const int4 w = a.items[it];
    const int dm = __builtin_amdgcn_readfirstlane(w.x);
    const DomainArgs d = a.doms[dm];
    const long long off = a.offs[dm];
    // after the loads it must not wait for (memory counters drain in order)
    const unsigned frozen = domain_frozen(a.status + dm);
    sweep_tile<CW, true>(d, a.src_buf + off, a.dst_buf + off, a.status + dm, a.rows,
                         __builtin_amdgcn_readfirstlane(w.y), __builtin_amdgcn_readfirstlane(w.z),
                         frozen, R);
  }
}

}  // namespace HLBM_NS
}  // namespace hlbm

#include "hlbm_step2.hpp"
#include "closure_device.hpp"  // the per-node correction the tile kernels can apply
#include "hlbm_tile.hpp"

namespace hlbm {
namespace HLBM_NS {

// ------------------------------------------------------ initialisation
//
// F0 = f^eq + f^1[a1FD] - psi/2 (algorithm of Sec. 3.5, steps 2-4), one
// thread per node, stencils read straight from the input fields.
struct InitArgs {
  DomainArgs d;
  const real *rho, *ux, *uy, *s;
  real *dst;  // ten planes
};

__device__ __forceinline__ void load_node(const InitArgs &a, int x, int y, real &r, real &u,
                                          real &v, real &th) {
  const int cx = map_index(x, a.d.nx, a.d.bcx), cy = map_index(y, a.d.ny, a.d.bcy);
  const long long i = (long long)cy * a.d.nx + cx;
  r = a.rho[i];
  u = a.ux[i];
  v = a.uy[i];
  // absolute entropy in: theta = rho^(gamma-1) exp(s / c_v)
  th = exp_r(a.s[i] * a.d.inv_cv + a.d.gm1 * log_r(r));
}

__global__ void k_init(InitArgs a) {
  const DomainArgs &d = a.d;
  const long long n = (long long)d.nx * d.ny;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % d.nx), y = (int)(i / d.nx);
    real rho, ux, uy, th, re, ue, ve, te, rw, uw, vw, tw, rn, un, vn, tn, rs, us, vs, ts;
    load_node(a, x, y, rho, ux, uy, th);
    load_node(a, x + 1, y, re, ue, ve, te);
    load_node(a, x - 1, y, rw, uw, vw, tw);
    load_node(a, x, y + 1, rn, un, vn, tn);
    load_node(a, x, y - 1, rs, us, vs, ts);
    const real cs2 = real(kCs2);
    const real dxux = real(0.5) * (ue - uw), dxuy = real(0.5) * (ve - vw);
    const real dyux = real(0.5) * (un - us), dyuy = real(0.5) * (vn - vs);
    const real div = dxux + dyuy;
    const real p = rho * cs2 * th;
    const real tau = d.mu / p, taub = tau + real(0.5);
    auto gam = [](real r, real u, real t) { return r * u * ((real(1) - t) - u * u); };
    const real gc = gam(rho, ux, th), gxe = gam(re, ue, te), gxw = gam(rw, uw, tw);
    const real gcy = gam(rho, uy, th), gyn = gam(rn, vn, tn), gys = gam(rs, vs, ts);
    real e1x, e1y;
    if (d.flags & kFlagE1Centred) {
      e1x = real(0.5) * (gxe - gxw);
      e1y = real(0.5) * (gyn - gys);
    } else {
      const real ep = d.sgn_eps;
      e1x = ux > ep ? gc - gxw : (ux < -ep ? gxe - gc : real(0.5) * (gxe - gxw));
      e1y = uy > ep ? gcy - gys : (uy < -ep ? gyn - gcy : real(0.5) * (gyn - gys));
    }
    const real e2 = (d.flags & kFlagE2Off) ? real(0) : d.e2c * p * div;
    const real Exx = e1x + e2, Eyy = e1y + e2;
    const real tp = taub * p;
    const real a1xx = -tp * (dxux - dyuy), a1yy = -a1xx, a1xy = -tp * (dyux + dxuy);
    const real c = cs2 * (th - real(1));
    const real a1xxy = uy * a1xx + real(2) * ux * a1xy;
    const real a1xyy = ux * a1yy + real(2) * uy * a1xy;
    const real a1xxyy = real(2) * (ux * a1xyy + uy * a1xxy) + (c - ux * ux) * a1yy +
                        (c - uy * uy) * a1xx - real(4) * ux * uy * a1xy;
    const real rc = rho * c;
    const real cref = cs2 * (d.theta_ref - real(1));
    const real A0 = rho - d.rho_ref;
    const real Axx = rho * ux * ux + (rc - d.rho_ref * cref) + a1xx - real(0.5) * Exx;
    const real Ayy = rho * uy * uy + (rc - d.rho_ref * cref) + a1yy - real(0.5) * Eyy;
    const real Axy = rho * ux * uy + a1xy;
    const real Axxy = rho * ux * ux * uy + rc * uy + a1xxy;
    const real Axyy = rho * ux * uy * uy + rc * ux + a1xyy;
    const real Axxyy = (d.flags & kFlagFeq3) ? real(0)
                                             : rho * ux * ux * uy * uy + rc * (ux * ux + uy * uy) +
                                                   (rc * c - d.rho_ref * cref * cref) + a1xxyy;
    real f[kQ];
    project(A0, rho * ux, rho * uy, Axx, Axy, Ayy, Axxy, Axyy, Axxyy, f);
    const long long P = d.plane;
    const long long o = (long long)y * d.pitch + x;
#pragma unroll
    for (int q = 0; q < kQ; ++q) a.dst[q * P + o] = f[q];
    a.dst[9 * P + o] = a.s[i] - d.s_ref;
  }
}

// ------------------------------------------------------------ walls
//
// Isothermal moving walls on the rows y = 0 and y = ny - 1 (bcy == kBcWall),
// a regularised wet-node wall: our reading of the wall condition that the
// thermal Couette case of Sec. 4.4 takes from an earlier paper without
// stating it.  After every step (and after initialisation) each wall node is
// rebuilt as f^eq(rho_w, U, 0, theta_w) + f^1[a1FD], psi taken as zero, with
//   rho_w = its c_y = 0 populations plus twice those that arrived from the
//           interior (no mass flux through the wall);
//   a1FD  from the velocity gradient at the wall: zero along it, one-sided
//         second order across it, (-3 u_w + 4 u_1 - u_2) / 2 over the new
//         velocities of the next two rows;
//   s_w   = c_v ln(theta_w / rho_w^(gamma - 1)).
// One thread per wall node, in place: a thread reads its node and two rows
// of the interior, which no thread writes (ny >= 4).
struct WallArgs {
  DomainArgs d;
  real *state;  // plane 0 of the current state
};

__device__ __forceinline__ void wall_node(const WallArgs &a, const int t) {
  const DomainArgs &d = a.d;
  const int side = t >= d.nx ? 1 : 0;
  const int x = t - side * d.nx;
  const int yw = side ? d.ny - 1 : 0, dir = side ? -1 : 1;
  const real U = side ? d.wall_u_hi : d.wall_u_lo;
  const long long P = d.plane;
  real *node = a.state + (long long)yw * d.pitch + x;
  real F[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) F[q] = node[q * P];
  // arrived from the interior: c_y = -1 (4, 7, 8) at y = 0, c_y = +1 (2, 5, 6) at the top;
  // the rest state's share of the sum is exactly rho_ref, so this is rho_w - rho_ref
  const real in = side ? (F[2] + F[5]) + F[6] : (F[4] + F[7]) + F[8];
  const real dr = ((F[0] + F[1]) + F[3]) + real(2) * in;
  const real rho = dr + d.rho_ref;
  auto velocity = [&](int y, real &ux, real &uy) {
    const real *p = a.state + (long long)y * d.pitch + x;
    real G[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) G[q] = p[q * P];
    const NodeMoments m = node_moments(G, d);
    ux = m.jx / m.rho;
    uy = m.jy / m.rho;
  };
  real u1x, u1y, u2x, u2y;
  velocity(yw + dir, u1x, u1y);
  velocity(yw + 2 * dir, u2x, u2y);
  const real half = real(0.5) * real(dir);
  const real dyux = half * ((real(4) * u1x - u2x) - real(3) * U);
  const real dyuy = half * (real(4) * u1y - u2y);
  const real cs2 = real(kCs2);
  const real th = d.wall_theta;
  const real p = rho * cs2 * th;
  const real tp = (d.mu / p + real(0.5)) * p;  // taubar p
  // a1FD = -taubar p (grad u + grad u^T - div I) with d/dx = 0 and div = dyuy
  const real a1xx = tp * dyuy, a1yy = -a1xx, a1xy = -tp * dyux;
  const real c = cs2 * (th - real(1));
  const real a1xxy = real(2) * U * a1xy;
  const real a1xyy = U * a1yy;
  const real a1xxyy = real(2) * U * a1xyy + (c - U * U) * a1yy + c * a1xx;
  // deviations from the rest reference formed from deviations (theta_w is
  // exact, so nothing cancels): rho c - rho_ref c_ref = (p - p_ref) - cs2
  // (rho - rho_ref), rho c^2 - rho_ref c_ref^2 = dr c^2 + rho_ref dc (c + c_ref)
  const real rc = rho * c;
  const real cref = cs2 * (d.theta_ref - real(1));
  const real dth = th - d.theta_ref;
  const real dp = cs2 * (dr * th + d.rho_ref * dth);
  const real drc = dp - cs2 * dr;
  const real drc2 = dr * c * c + d.rho_ref * (cs2 * dth) * (c + cref);
  const real Axx = rho * U * U + drc + a1xx;
  const real Ayy = drc + a1yy;
  const real Axy = a1xy;
  const real Axxy = a1xxy;
  const real Axyy = rc * U + a1xyy;
  const real Axxyy = (d.flags & kFlagFeq3) ? real(0) : rc * U * U + drc2 + a1xxyy;
  real f[kQ];
  project(dr, rho * U, real(0), Axx, Axy, Ayy, Axxy, Axyy, Axxyy, f);
#pragma unroll
  for (int q = 0; q < kQ; ++q) node[q * P] = f[q];
  // s_w - s_ref = c_v (ln(theta_w / theta_ref) - (gamma - 1) ln(rho_w / rho_ref))
  node[9 * P] = (log_r(th) - log_r(d.theta_ref) - d.gm1 * (log_r(rho) - d.log_rho_ref)) / d.inv_cv;
}

__global__ void k_wall(WallArgs a) {
  const int n = 2 * a.d.nx;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    wall_node(a, t);
}

// ------------------------------------------------------------ moments
struct FieldArgs {
  DomainArgs d;
  const real *state;
  real *rho, *ux, *uy, *s, *theta;
};

__global__ void k_moments(FieldArgs a) {
  const DomainArgs &d = a.d;
  const long long n = (long long)d.nx * d.ny, P = d.plane;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long o = state_off(d, i);
    real F[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) F[q] = a.state[q * P + o];
    const real sv = a.state[9 * P + o];
    const NodeMoments m = node_moments(F, d);
    if (a.rho) a.rho[i] = m.rho;
    if (a.ux) a.ux[i] = m.jx / m.rho;
    if (a.uy) a.uy[i] = m.jy / m.rho;
    if (a.s) a.s[i] = sv + d.s_ref;
    if (a.theta) a.theta[i] = node_theta(m.rho, sv, d);
  }
}

// Absolute populations out / in.
struct PopArgs {
  DomainArgs d;
  real *state;
  real *F9;
  real *s;
  int to_state;
};

__global__ void k_populations(PopArgs a) {
  const DomainArgs &d = a.d;
  const long long n = (long long)d.nx * d.ny, P = d.plane;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long o = state_off(d, i);
    if (a.to_state) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) a.state[q * P + o] = a.F9[q * n + i] - d.fref[q];
      a.state[9 * P + o] = a.s[i] - d.s_ref;
    } else {
#pragma unroll
      for (int q = 0; q < kQ; ++q) a.F9[q * n + i] = a.state[q * P + o] + d.fref[q];
    }
  }
}

// ------------------------------------------------------- reductions
// Per-workgroup FP64 partials of {mass, mom x, mom y, energy, bad, max CFL}.
constexpr int kRedThreads = 256;
constexpr int kRedVals = 6;

struct ReduceArgs {
  DomainArgs d;
  const real *state;
  double *partials;  // [gridDim.x][kRedVals]
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__global__ __launch_bounds__(kRedThreads) void k_reduce(ReduceArgs a) {
  const DomainArgs &d = a.d;
  const long long n = (long long)d.nx * d.ny, P = d.plane;
  const double cv = kCs2 / (double)d.gm1;
  double acc[kRedVals] = {0, 0, 0, 0, 0, 0};
  // Fixed per-thread assignment and fixed combine order: deterministic.
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < n;
       i += (long long)gridDim.x * kRedThreads) {
    const long long o = state_off(d, i);
    real F[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) F[q] = a.state[q * P + o];
    const real sv = a.state[9 * P + o];
    const NodeMoments m = node_moments(F, d);
    const double rho = (double)m.rho;
    const double ux = (double)m.jx / rho, uy = (double)m.jy / rho;
    const double th = (double)node_theta(m.rho, sv, d);
    acc[0] += rho;
    acc[1] += (double)m.jx;
    acc[2] += (double)m.jy;
    acc[3] += rho * cv * th + 0.5 * rho * (ux * ux + uy * uy);
    const bool ok = rho > 0.0 && th > 0.0 && __builtin_isfinite(ux + uy + th + (double)sv);
    acc[4] += ok ? 0.0 : 1.0;
    const double cfl = ok ? sqrt(ux * ux + uy * uy) + sqrt((double)d.gamma * kCs2 * th) : 0.0;
    acc[5] = fmax(acc[5], cfl);
  }
  __shared__ double sm[kRedThreads / 64][kRedVals];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kRedVals; ++k) {
    const double v = k == 5 ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) sm[w][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kRedVals) {
    const int k = threadIdx.x;
    double v = sm[0][k];
    for (int ww = 1; ww < kRedThreads / 64; ++ww) v = k == 5 ? fmax(v, sm[ww][k]) : v + sm[ww][k];
    a.partials[(long long)blockIdx.x * kRedVals + k] = v;
  }
}

// Second pass: one workgroup combines the partials in a fixed order.
__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double *partials, int nparts,
                                                              double *out) {
  double acc[kRedVals] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += kRedThreads) {
#pragma unroll
    for (int k = 0; k < kRedVals; ++k) {
      const double v = partials[(long long)b * kRedVals + k];
      acc[k] = k == 5 ? fmax(acc[k], v) : acc[k] + v;
    }
  }
  __shared__ double sm[kRedThreads / 64][kRedVals];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kRedVals; ++k) {
    const double v = k == 5 ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) sm[w][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kRedVals) {
    const int k = threadIdx.x;
    double v = sm[0][k];
    for (int ww = 1; ww < kRedThreads / 64; ++ww) v = k == 5 ? fmax(v, sm[ww][k]) : v + sm[ww][k];
    out[k] = v;
  }
}

// s = c_v ln(theta / rho^(gamma-1)).
__global__ void k_entropy(const real *rho, const real *theta, real *s, long long n, real inv_cv,
                          real gm1) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    s[i] = (log_r(theta[i]) - gm1 * log_r(rho[i])) / inv_cv;
  }
}

}  // namespace HLBM_NS
}  // namespace hlbm
