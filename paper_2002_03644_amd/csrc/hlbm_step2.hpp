// Two time steps per sweep: the fused step applied twice inside one pass over
// the state, for domains periodic along both axes (included at the end of
// hlbm_device.hpp).
//
// The one-step sweep reads the ten planes once and writes them once per
// step; its arithmetic runs far below the chip's VALU rate (doubling it costs
// 0-6 % of the step time), so the step is bound by the state traffic.  Here
// a workgroup reads the state at level n once and writes level n + 2 once:
// the per-node arithmetic of each step is the one-step kernel's, in the
// same order (FP64 results are bitwise those of two single steps), and level
// n + 1 lives only in registers and LDS rings.
//
// Geometry.  Output tile: CW columns from x0, `rows` rows from y0.  Level
// n + 2 there needs level n + 1 on a radius-2 halo (CW + 4 columns, rows + 4
// rows), which needs level n on a radius-4 halo: CW + 8 columns, rows + 8
// rows.  Lanes 0..CW-1 hold the tile's columns (aligned loads and stores),
// lanes CW..CW+7 the four halo columns on each side; the rest of the last
// wave only joins the barriers.  A column's ring position is ri = column -
// (x0 - 4).  Virtual row j is grid row y0 - 4 + j.
//
// Stages per level (A: moments into the rings, B: collision, C: streaming and
// entropy, as in the one-step sweep), on the ring positions that have their
// stencils: A1 on 0..CW+7, B1 on 1..CW+6, C1 on 2..CW+5; C1's output (the
// nine populations and the entropy of level n + 1 at the lane's own node)
// feeds A2 in registers on the same lanes; B2 on 3..CW+4; C2 on the tile.
// Iteration i issues the loads of row i + 1, runs B1(i - 1) and B2(i - 4),
// a barrier, A1(i + 1), C1(i - 2) -> A2(i - 2), C2(i - 5), a barrier.  Each
// level keeps the one-step sweep's distances between A, B and C, so its
// rings have the same depths, except those of s and theta (see LevelRings):
// C takes their y-stencil from per-lane registers, which leaves 26 rows of
// CW + 8 per level in LDS, so four workgroups of 184-column tiles (three
// whole waves each) fit a compute unit.
//
// Boundaries: out-of-range columns and rows wrap.  A halo lane then computes
// level n + 1 of the wrapped node from the wrapped stencil, bit for bit what
// the node's own lane computes, so periodic domains of any size (including
// ragged tiles and grids thinner than the halo) are exact.  Clamped
// boundaries would need the ghost copies of level n + 1, which this sweep
// does not form; they and walls take the one-step kernel.
#pragma once

namespace hlbm {
namespace HLBM_NS {

// LDS rings of one time level (the depths of the one-step sweep's rings,
// except s and theta: C reads them from LDS only along x, on its own row,
// and takes the y-stencil from the lane's register window, so four rows
// hold every row still to be read).
template <int W>
struct LevelRings {
  real ux[2][W], uy[2][W], gx[2][W];
  real th[4][W], s[4][W];
  real f0[2][2][W];  // populations 1, 3   (c_y =  0)
  real fp[3][2][W];  // populations 5, 6   (c_y = +1)
  real fm[2][W];     // populations 7, 8   (c_y = -1)
};

template <int CW>
struct TileRings2 {
  static constexpr int W = CW + 8;
  LevelRings<W> L1, L2;
};

// Threads of a two-step workgroup: the tile's CW columns and the 8 halo
// columns, rounded up to whole waves.
constexpr int step2_threads(int cw) { return (cw + 8 + 63) / 64 * 64; }

// Per-lane registers of one time level: the node state of rows k and k + 1
// carried from A to B, B's y-stencil along the lane's column, and the B -> C
// carries with populations 0, 2 and 4 (see the one-step sweep).
struct LevelRegs {
  real s0_dr = 0, s0_rho = 1, s0_pxx = 0, s0_pyy = 0, s0_pxy = 0, s0_ux = 0, s0_uy = 0, s0_th = 1;
  real s1_dr = 0, s1_rho = 1, s1_pxx = 0, s1_pyy = 0, s1_pxy = 0, s1_ux = 0, s1_uy = 0, s1_th = 1;
  real m_ux = 0, m_uy = 0, m_gy = 0, c_gy = 0, n_gy = 0;
  real nB_ux = 0, nB_uy = 0, nB_rho = 1, nB_th = 1, nB_phi = 0;
  real cB_ux = 0, cB_uy = 0, cB_rho = 1, cB_th = 1, cB_phi = 0;
  real nB_f0 = 0, nB_f2 = 0, nB_f4 = 0, cB_f0 = 0, cB_f2 = 0, cB_f2b = 0;
  // the lane's own column of s and of the theta values C's Laplacian reads,
  // over the last six (five) rows A wrote, oldest first: C(k) runs after
  // A(k + 3) and reads rows k - 2 .. k + 2 (k - 1 .. k + 1)
  real ws[6] = {0, 0, 0, 0, 0, 0};
  real wt[5] = {0, 0, 0, 0, 0};
};

// Shifts one row into the register windows (level_a does it for the row it
// writes; a lane whose A stage has run out pushes a placeholder, so the
// windows stay aligned with C's rows).
__device__ __forceinline__ void level_push(LevelRegs &g, const real sv, const real lap_val) {
#pragma unroll
  for (int q = 0; q < 5; ++q) g.ws[q] = g.ws[q + 1];
  g.ws[5] = sv;
#pragma unroll
  for (int q = 0; q < 4; ++q) g.wt[q] = g.wt[q + 1];
  g.wt[4] = lap_val;
}

// A(j): moments of one node of row j from its nine populations and entropy.
template <int W>
__device__ __forceinline__ void level_a(const DomainArgs &d, LevelRegs &g, LevelRings<W> &R,
                                        const int j, const int ri, const real (&F)[kQ],
                                        const real sv, unsigned &bad) {
  const NodeMoments m = node_moments(F, d);
  const real inv_rho = rcp_fast(m.rho);
  const real ux = m.jx * inv_rho, uy = m.jy * inv_rho;
  real th, lap_val;
  if (d.flags & kFlagPreciseTheta) {
    lap_val = node_dtheta(m.dr, m.rho, sv, d);
    th = d.theta_ref + lap_val;
  } else {
    th = node_theta(m.rho, sv, d);
    lap_val = th;
  }
  R.ux[j & 1][ri] = ux;
  R.uy[j & 1][ri] = uy;
  R.th[j & 3][ri] = lap_val;
  R.gx[j & 1][ri] = m.rho * ux * ((real(1) - th) - ux * ux);
  R.s[j & 3][ri] = sv;
  level_push(g, sv, lap_val);
  g.m_ux = g.s0_ux;
  g.m_uy = g.s0_uy;
  g.m_gy = g.c_gy;
  g.c_gy = g.n_gy;
  g.n_gy = m.rho * uy * ((real(1) - th) - uy * uy);
  g.s0_dr = g.s1_dr;
  g.s0_rho = g.s1_rho;
  g.s0_pxx = g.s1_pxx;
  g.s0_pyy = g.s1_pyy;
  g.s0_pxy = g.s1_pxy;
  g.s0_ux = g.s1_ux;
  g.s0_uy = g.s1_uy;
  g.s0_th = g.s1_th;
  g.s1_dr = m.dr;
  g.s1_rho = m.rho;
  g.s1_pxx = m.pxx;
  g.s1_pyy = m.pyy;
  g.s1_pxy = m.pxy;
  g.s1_ux = ux;
  g.s1_uy = uy;
  g.s1_th = th;
  bad |= (m.rho > real(0) && th > real(0) && __builtin_isfinite(ux + uy + th)) ? 0u : 1u;
}

// B(k): gradients, correction term, HRR stress and the nine post-collision
// populations of row k (row k + 1 was the last A).
template <int W>
__device__ __forceinline__ void level_b(const DomainArgs &d, LevelRegs &g, LevelRings<W> &R,
                                        const int k, const int ri) {
  const real cs2 = real(kCs2);
  const real cref = cs2 * (d.theta_ref - real(1));
  const int sc = k % 3;
  const real rho = g.s0_rho, ux = g.s0_ux, uy = g.s0_uy, th = g.s0_th;
  const int su = k & 1;
  const real uxe = R.ux[su][ri + 1], uxw = R.ux[su][ri - 1];
  const real uye = R.uy[su][ri + 1], uyw = R.uy[su][ri - 1];
  const real uxn = g.s1_ux, uxs = g.m_ux;
  const real uyn = g.s1_uy, uys = g.m_uy;
  const real dxux = real(0.5) * (uxe - uxw), dxuy = real(0.5) * (uye - uyw);
  const real dyux = real(0.5) * (uxn - uxs), dyuy = real(0.5) * (uyn - uys);
  const real div = dxux + dyuy;
  const real p = rho * cs2 * th;
  const real dth = th - d.theta_ref;
  const real dp = cs2 * (g.s0_dr * th + d.rho_ref * dth);  // p - p_ref
  const real tau = div_fast(d.mu, p);
  const real taub = tau + real(0.5);
  const real itaub = rcp_fast(taub);
  const real gc = R.gx[k & 1][ri];
  const real gxe = R.gx[k & 1][ri + 1], gxw = R.gx[k & 1][ri - 1];
  const real gcy = g.c_gy;
  const real gyn = g.n_gy, gys = g.m_gy;
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
  const real rux = rho * ux, ruy = rho * uy;
  const real ruxx = rux * ux, ruyy = ruy * uy, ruxy = rux * uy;
  const real prxx = (g.s0_pxx - dp) - ruxx + real(0.5) * Exx;
  const real pryy = (g.s0_pyy - dp) - ruyy + real(0.5) * Eyy;
  const real prxy = g.s0_pxy - ruxy;
  const real tp = taub * p;
  const real fdxx = -tp * (dxux - dyuy);
  const real fdxy = -tp * (dyux + dxuy);
  const real sg = d.sigma, sg1 = real(1) - sg;
  const real a1xx = sg * prxx + sg1 * fdxx;
  const real a1yy = sg * pryy - sg1 * fdxx;
  const real a1xy = sg * prxy + sg1 * fdxy;
  const real c = cs2 * (th - real(1));
  const real a1xxy = uy * a1xx + real(2) * ux * a1xy;
  const real a1xyy = ux * a1yy + real(2) * uy * a1xy;
  const real a1xxyy = real(2) * (ux * a1xyy + uy * a1xxy) + (c - ux * ux) * a1yy +
                      (c - uy * uy) * a1xx - real(4) * ux * uy * a1xy;
  const real om = real(1) - itaub;
  const real drc = dp - cs2 * g.s0_dr;
  const real dc = cs2 * dth;
  const real drc2 = g.s0_dr * c * c + d.rho_ref * dc * (c + cref);
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
  project(g.s0_dr, rux, ruy, Axx, Axy, Ayy, Axxy, Axyy, Axxyy, f);
  R.f0[k & 1][0][ri] = f[1];
  R.f0[k & 1][1][ri] = f[3];
  R.fp[sc][0][ri] = f[5];
  R.fp[sc][1][ri] = f[6];
  R.fm[0][ri] = f[7];
  R.fm[1][ri] = f[8];
  g.nB_f0 = f[0];
  g.nB_f2 = f[2];
  g.nB_f4 = f[4];
  real phi;
  if (d.flags & kFlagPhiFD) {
    const real aa = dxux - dyuy, bb = dyux + dxuy;
    phi = d.mu * (aa * aa + bb * bb);
  } else {
    phi = -(tau * itaub) * (a1xx * dxux + a1xy * (dyux + dxuy) + a1yy * dyuy);
  }
  g.nB_ux = ux;
  g.nB_uy = uy;
  g.nB_rho = rho;
  g.nB_th = th;
  g.nB_phi = phi;
}

// C(k): pull streaming of row k and its entropy update (B(k + 1) has run).
template <int W>
__device__ __forceinline__ void level_c(const DomainArgs &d, const LevelRegs &g,
                                        LevelRings<W> &R, const int k, const int ri,
                                        real (&Fo)[kQ], real &snew) {
  const int z = k & 1, pm = (k + 2) % 3;
  Fo[0] = g.cB_f0;
  Fo[1] = R.f0[z][0][ri - 1];
  Fo[3] = R.f0[z][1][ri + 1];
  Fo[2] = g.cB_f2b;
  Fo[5] = R.fp[pm][0][ri - 1];
  Fo[6] = R.fp[pm][1][ri + 1];
  Fo[4] = g.nB_f4;
  Fo[7] = R.fm[0][ri + 1];
  Fo[8] = R.fm[1][ri - 1];
  const int s0 = k & 3;
  const real sc = g.ws[2];
  const real advx = muscl_term(g.cB_ux, R.s[s0][ri - 2], R.s[s0][ri - 1], sc, R.s[s0][ri + 1],
                               R.s[s0][ri + 2]);
  const real advy = muscl_term(g.cB_uy, g.ws[0], g.ws[1], sc, g.ws[3], g.ws[4]);
  const real lap = ((R.th[s0][ri + 1] + R.th[s0][ri - 1]) + (g.wt[2] + g.wt[0])) -
                   real(4) * g.wt[1];
  snew = sc - (advx + advy) + div_fast(d.lambda * lap + g.cB_phi, g.cB_rho * g.cB_th);
}

// End of an iteration: B's results move to the C carries.
__device__ __forceinline__ void level_advance(LevelRegs &g) {
  g.cB_ux = g.nB_ux;
  g.cB_uy = g.nB_uy;
  g.cB_rho = g.nB_rho;
  g.cB_th = g.nB_th;
  g.cB_phi = g.nB_phi;
  g.cB_f2b = g.cB_f2;
  g.cB_f2 = g.nB_f2;
  g.cB_f0 = g.nB_f0;
}

template <int CW, bool kBatch = false>
__device__ __forceinline__ void sweep_tile2(const DomainArgs &d, const real *src0, real *dst0,
                                            unsigned *status, const int rows, const int bx,
                                            const int by, const unsigned frozen,
                                            TileRings2<CW> &R) {
  const int t = threadIdx.x;
  const real *src[kPlanes];
  real *dst[kPlanes];
#pragma unroll
  for (int q = 0; q < kPlanes; ++q) {
    src[q] = src0 + (long long)q * d.plane;
    dst[q] = dst0 + (long long)q * d.plane;
  }
  const int x0 = bx * CW, y0 = by * rows;
  // lane -> ring position: tile lanes at 4..CW+3, halo lanes at 0..3 and CW+4..CW+7
  const int h = t - CW;
  const bool a1 = t < CW + 8;
  const int ri = t < CW ? t + 4 : (h < 4 ? h : (h < 8 ? CW + h : 0));
  const bool b1 = a1 && ri >= 1 && ri <= CW + 6;
  const bool c1 = a1 && ri >= 2 && ri <= CW + 5;   // these lanes also run A2
  const bool b2 = a1 && ri >= 3 && ri <= CW + 4;
  const int vx = x0 - 4 + ri;
  const bool c2 = t < CW && vx < d.nx;
  const int cx = map_index(vx, d.nx, d.bcx);
  const int nrow = min(rows, d.ny - y0);
  const int nit = nrow + 9;
  constexpr unsigned kEl = sizeof(real);
  unsigned bad = 0;
  LevelRegs g1, g2;

  auto row_off = [&](int j) {
    return (unsigned)(map_index(y0 - 4 + j, d.ny, d.bcy) * d.pitch + cx) * kEl;
  };

  if (a1) {  // prologue: A1(0)
    real F[kQ];
    const unsigned off = row_off(0);
#pragma unroll
    for (int q = 0; q < kQ; ++q) F[q] = load_at(src[q], off);
    level_a(d, g1, R.L1, 0, ri, F, load_at(src[9], off), bad);
  }
  if (barrier_skip<kBatch>(frozen)) return;

  for (int i = 0; i < nit; ++i) {
    // ---------------- loads of row i + 1 (consumed by A1 after the B stages)
    real ld[kPlanes];
    const bool do_a = a1 && i + 1 <= nrow + 7;
    if (do_a) {
      const unsigned off = row_off(i + 1);
#pragma unroll
      for (int q = 0; q < kPlanes; ++q) ld[q] = load_at(src[q], off);
    }
    // ---------------- B1(i - 1), B2(i - 4)
    if (b1 && i >= 2 && i - 1 <= nrow + 6) level_b(d, g1, R.L1, i - 1, ri);
    if (b2 && i >= 7 && i - 4 <= nrow + 4) level_b(d, g2, R.L2, i - 4, ri);
    __syncthreads();

    // ---------------- A1(i + 1), C1(i - 2) -> A2(i - 2), C2(i - 5)
    if (do_a) {
      real F[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) F[q] = ld[q];
      level_a(d, g1, R.L1, i + 1, ri, F, ld[9], bad);
    } else if (a1) {
      level_push(g1, real(0), real(0));
    }
    if (c1 && i >= 4 && i - 2 <= nrow + 5) {
      real Fo[kQ], snew;
      level_c(d, g1, R.L1, i - 2, ri, Fo, snew);
      level_a(d, g2, R.L2, i - 2, ri, Fo, snew, bad);
    } else if (c1 && i >= 4) {
      level_push(g2, real(0), real(0));
    }
    if (c2 && i >= 9) {
      const int k = i - 5;
      real Fo[kQ], snew;
      level_c(d, g2, R.L2, k, ri, Fo, snew);
      const unsigned off = (unsigned)((y0 + k - 4) * d.pitch + vx) * kEl;
#pragma unroll
      for (int q = 0; q < kQ; ++q) store_stream(dst[q], off, Fo[q]);
      store_stream(dst[9], off, snew);
    }
    level_advance(g1);
    level_advance(g2);
    __syncthreads();
  }
  if (bad) atomicOr(status, 1u);
}

// Two steps of a whole periodic domain: one workgroup per tile.
template <int CW>
__global__ __launch_bounds__(step2_threads(CW)) void k_step2(StepArgs a) {
  __shared__ TileRings2<CW> R;
  int bid = blockIdx.x;
  const int nblk = a.nbx * a.nby;
  if (a.xcd_remap) {
    const int per = (nblk + 7) >> 3;
    const int xcd = bid & 7, k = bid >> 3;
    const int full = nblk - (per - 1) * 8;
    bid = xcd < full ? xcd * per + k : full * per + (xcd - full) * (per - 1) + k;
  }
  sweep_tile2<CW>(a.d, a.src, a.dst, a.status, a.rows, bid % a.nbx, bid / a.nbx, 0, R);
}

// Two steps of a batch of periodic domains: the persistent walk over (domain,
// tile) items of the one-step batch kernel, with the two-step sweep.
template <int CW>
__global__ __launch_bounds__(step2_threads(CW)) void k_step_batch2(BatchArgs a) {
  __shared__ TileRings2<CW> R;
  const TileWalk walk = tile_walk(a.nitems, a.xcd_walk);
  for (int it = walk.first; it < walk.end; it += walk.step) {
    const int4 w = a.items[it];
    const int dm = __builtin_amdgcn_readfirstlane(w.x);
    const DomainArgs d = a.doms[dm];
    const long long off = a.offs[dm];
    // after the loads it must not wait for (memory counters drain in order)
    const unsigned frozen = domain_frozen(a.status + dm);
    sweep_tile2<CW, true>(d, a.src_buf + off, a.dst_buf + off, a.status + dm, a.rows,
                          __builtin_amdgcn_readfirstlane(w.y),
                          __builtin_amdgcn_readfirstlane(w.z), frozen, R);
  }
}

}  // namespace HLBM_NS
}  // namespace hlbm
