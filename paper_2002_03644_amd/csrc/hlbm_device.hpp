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
  int flags;           // bit 0: Phi by finite differences, bit 1: centred E1, bit 2: no E2
  real mu, sigma, lambda, inv_cv, gm1, e2c, gamma, sgn_eps;
  real rho_ref, theta_ref, log_rho_ref, s_ref;
  real fref[kQ];       // deviation reference populations (zero in the FP64 form)
};

struct StepArgs {
  DomainArgs d;
  const real *__restrict__ src;
  real *__restrict__ dst;
  unsigned *status;    // bit 0 set when a node diverged
  int rows;            // output rows per strip
  int ow;              // output columns per workgroup (tile width - 4)
  int nbx, nby;        // workgroups along x and y
  int xcd_remap;       // 1: spread spatial neighbours onto the same XCD
};

constexpr int kFlagPhiFD = 1, kFlagE1Centred = 2, kFlagE2Off = 4;

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
// One workgroup owns a strip of `ow = BW - 4` output columns and `rows` output
// rows.  Thread t handles virtual column x0 - 2 + t and sweeps the rows of the
// strip; per row j of the sweep:
//   A(j)    loads the ten planes at row j (prefetched one row ahead) and puts
//           u, theta, Gamma and s of the node into LDS rings;
//   B(j-1)  builds gradients, E, a1 and the nine post-collision populations of
//           row j-1 (radius-1 stencil through the rings) into an LDS ring;
//   C(j-2)  pull-streams the populations of row j-2 out of that ring and
//           updates its entropy (radius-2 stencil), storing both.
// Each node's moments and collision are therefore computed once per step
// (plus a 4-column halo), and HBM sees one read and one write of the state.
template <int BW>
__global__ __launch_bounds__(BW) void k_step(StepArgs a) {
  constexpr int R = 6;   // rows kept of the moment rings (C reads rows j-4..j)
  __shared__ real r_ux[R][BW], r_uy[R][BW], r_th[R][BW], r_gx[R][BW], r_gy[R][BW], r_s[R][BW];
  __shared__ real r_f[3][kQ][BW];

  const DomainArgs &d = a.d;
  const int t = threadIdx.x;
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
  const int bx = bid % a.nbx, by = bid / a.nbx;
  const int x0 = bx * a.ow, y0 = by * a.rows;
  const int vx = x0 - 2 + t;
  const int cx = map_index(vx, d.nx, d.bcx);
  const int nrow = min(a.rows, d.ny - y0);
  const int nit = nrow + 4;
  const long long P = d.plane;
  const bool own_col = (t >= 2) && (t < BW - 2) && (vx < d.nx);
  const bool b_col = (t >= 1) && (t < BW - 1);
  const real cs2 = real(kCs2);
  const real cref = cs2 * (d.theta_ref - real(1));

  // prefetch row 0
  real ld[kPlanes];
  {
    const int ry = map_index(y0 - 2, d.ny, d.bcy);
    const real *p = a.src + (long long)ry * d.nx + cx;
#pragma unroll
    for (int q = 0; q < kPlanes; ++q) ld[q] = p[q * P];
  }

  // A -> B carry (node state of the row last loaded)
  real nA_dr = 0, nA_rho = 1, nA_pxx = 0, nA_pyy = 0, nA_pxy = 0, nA_ux = 0, nA_uy = 0, nA_th = 1;
  // B -> C carry
  real nB_ux = 0, nB_uy = 0, nB_rho = 1, nB_th = 1, nB_phi = 0;
  unsigned bad = 0;

  for (int j = 0; j < nit; ++j) {
    const real cA_dr = nA_dr, cA_rho = nA_rho, cA_pxx = nA_pxx, cA_pyy = nA_pyy,
               cA_pxy = nA_pxy, cA_ux = nA_ux, cA_uy = nA_uy, cA_th = nA_th;
    const real cB_ux = nB_ux, cB_uy = nB_uy, cB_rho = nB_rho, cB_th = nB_th, cB_phi = nB_phi;

    // ---------------- A(j): moments of row j
    {
      real F[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) F[q] = ld[q];
      const real sv = ld[9];
      if (j + 1 < nit) {
        const int ry = map_index(y0 - 1 + j, d.ny, d.bcy);
        const real *p = a.src + (long long)ry * d.nx + cx;
#pragma unroll
        for (int q = 0; q < kPlanes; ++q) ld[q] = p[q * P];
      }
      const NodeMoments m = node_moments(F, d);
      const real inv_rho = rcp_fast(m.rho);
      const real ux = m.jx * inv_rho, uy = m.jy * inv_rho;
      const real th = node_theta(m.rho, sv, d);
      const int sl = j % R;
      r_ux[sl][t] = ux;
      r_uy[sl][t] = uy;
      r_th[sl][t] = th;
      r_gx[sl][t] = m.rho * ux * ((real(1) - th) - ux * ux);
      r_gy[sl][t] = m.rho * uy * ((real(1) - th) - uy * uy);
      r_s[sl][t] = sv;
      nA_dr = m.dr;
      nA_rho = m.rho;
      nA_pxx = m.pxx;
      nA_pyy = m.pyy;
      nA_pxy = m.pxy;
      nA_ux = ux;
      nA_uy = uy;
      nA_th = th;
      bad |= (m.rho > real(0) && th > real(0) && __builtin_isfinite(ux + uy + th)) ? 0u : 1u;
    }
    __syncthreads();

    // ---------------- B(j-1): collision of row k = j-1
    if (j >= 2) {
      const int k = j - 1;
      const int sc = k % R, sn = (k + 1) % R, ss = (k + R - 1) % R;
      if (b_col) {
        const real rho = cA_rho, ux = cA_ux, uy = cA_uy, th = cA_th;
        const real uxe = r_ux[sc][t + 1], uxw = r_ux[sc][t - 1];
        const real uye = r_uy[sc][t + 1], uyw = r_uy[sc][t - 1];
        const real uxn = r_ux[sn][t], uxs = r_ux[ss][t];
        const real uyn = r_uy[sn][t], uys = r_uy[ss][t];
        const real dxux = real(0.5) * (uxe - uxw), dxuy = real(0.5) * (uye - uyw);
        const real dyux = real(0.5) * (uxn - uxs), dyuy = real(0.5) * (uyn - uys);
        const real div = dxux + dyuy;
        const real p = rho * cs2 * th;
        const real dth = th - d.theta_ref;
        const real dp = cs2 * (cA_dr * th + d.rho_ref * dth);  // p - p_ref
        const real tau = div_fast(d.mu, p);
        const real taub = tau + real(0.5);
        const real itaub = rcp_fast(taub);
        // E1 (upwind in the sign of the node velocity; centred when u = 0)
        const real gc = r_gx[sc][t];
        const real gxe = r_gx[sc][t + 1], gxw = r_gx[sc][t - 1];
        const real gcy = r_gy[sc][t];
        const real gyn = r_gy[sn][t], gys = r_gy[ss][t];
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
        const real prxx = (cA_pxx - dp) - ruxx + real(0.5) * Exx;
        const real pryy = (cA_pyy - dp) - ruyy + real(0.5) * Eyy;
        const real prxy = cA_pxy - ruxy;
        const real tp = taub * p;
        const real fdxx = -tp * (dxux - dyuy);
        const real fdxy = -tp * (dyux + dxuy);
        const real sg = d.sigma, sg1 = real(1) - d.sigma;
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
        const real drc = dp - cs2 * cA_dr;
        const real dc = cs2 * dth;
        const real drc2 = cA_dr * c * c + d.rho_ref * dc * (c + cref);
        const real Axx = ruxx + drc + om * a1xx + real(0.5) * Exx;
        const real Ayy = ruyy + drc + om * a1yy + real(0.5) * Eyy;
        const real Axy = ruxy + om * a1xy;
        const real rc = rho * c;
        const real Axxy = ruxx * uy + rc * uy + om * a1xxy;
        const real Axyy = ruyy * ux + rc * ux + om * a1xyy;
        const real Axxyy = ruxx * uy * uy + rc * (ux * ux + uy * uy) + drc2 + om * a1xxyy;
        real f[kQ];
        project(cA_dr, rux, ruy, Axx, Axy, Ayy, Axxy, Axyy, Axxyy, f);
        const int fs = k % 3;
#pragma unroll
        for (int q = 0; q < kQ; ++q) r_f[fs][q][t] = f[q];
        real phi;
        if (d.flags & kFlagPhiFD) {
          const real a = dxux - dyuy, b = dyux + dxuy;
          phi = d.mu * (a * a + b * b);
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

    // ---------------- C(j-2): stream and entropy of row k = j-2
    if (j >= 4) {
      const int k = j - 2;
      if (own_col) {
        const int f0 = k % 3, fm = (k + 2) % 3, fp = (k + 1) % 3;  // rows k, k-1, k+1
        real Fo[kQ];
        Fo[0] = r_f[f0][0][t];
        Fo[1] = r_f[f0][1][t - 1];
        Fo[2] = r_f[fm][2][t];
        Fo[3] = r_f[f0][3][t + 1];
        Fo[4] = r_f[fp][4][t];
        Fo[5] = r_f[fm][5][t - 1];
        Fo[6] = r_f[fm][6][t + 1];
        Fo[7] = r_f[fp][7][t + 1];
        Fo[8] = r_f[fp][8][t - 1];
        const int s0 = k % R, s1 = (k + 1) % R, s2 = (k + 2) % R, sm1 = (k + R - 1) % R,
                  sm2 = (k + R - 2) % R;
        const real sc = r_s[s0][t];
        const real advx = muscl_term(cB_ux, r_s[s0][t - 2], r_s[s0][t - 1], sc, r_s[s0][t + 1],
                                     r_s[s0][t + 2]);
        const real advy = muscl_term(cB_uy, r_s[sm2][t], r_s[sm1][t], sc, r_s[s1][t], r_s[s2][t]);
        const real lap = ((r_th[s0][t + 1] + r_th[s0][t - 1]) + (r_th[s1][t] + r_th[sm1][t])) -
                         real(4) * cB_th;
        const real snew = sc - (advx + advy) + div_fast(d.lambda * lap + cB_phi, cB_rho * cB_th);
        const int oy = y0 + k - 2;
        real *o = a.dst + (long long)oy * d.nx + vx;
#pragma unroll
        for (int q = 0; q < kQ; ++q) o[q * P] = Fo[q];
        o[9 * P] = snew;
      }
    }
  }
  if (bad) atomicOr(a.status, 1u);
}

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
    const real Axxyy = rho * ux * ux * uy * uy + rc * (ux * ux + uy * uy) +
                       (rc * c - d.rho_ref * cref * cref) + a1xxyy;
    real f[kQ];
    project(A0, rho * ux, rho * uy, Axx, Axy, Ayy, Axxy, Axyy, Axxyy, f);
    const long long P = d.plane;
    const long long o = (long long)y * d.nx + x;
#pragma unroll
    for (int q = 0; q < kQ; ++q) a.dst[q * P + o] = f[q];
    a.dst[9 * P + o] = a.s[i] - d.s_ref;
  }
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
    real F[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) F[q] = a.state[q * P + i];
    const real sv = a.state[9 * P + i];
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
    if (a.to_state) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) a.state[q * P + i] = a.F9[q * n + i] - d.fref[q];
      a.state[9 * P + i] = a.s[i] - d.s_ref;
    } else {
#pragma unroll
      for (int q = 0; q < kQ; ++q) a.F9[q * n + i] = a.state[q * P + i] + d.fref[q];
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
    real F[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) F[q] = a.state[q * P + i];
    const real sv = a.state[9 * P + i];
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
