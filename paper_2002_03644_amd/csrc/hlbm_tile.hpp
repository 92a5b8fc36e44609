// One step on two-dimensional tiles, for batches of small domains (included
// by hlbm_device.hpp after the row sweeps).
//
// The row sweeps pipeline a strip of rows through the stages; each strip
// reads rows + 4 input rows and pays a serial fill of the pipeline.  A 256^2
// domain cut into enough strips to fill the chip has strips of four rows:
// eight input rows for four output rows, and every wave runs every stage of
// every row, halo lanes included.  This kernel loads a TW x TH tile and its
// radius-2 halo at once and runs the stages over the whole tile, with a
// barrier between them:
//   A  moments of the tile, of the collision ring around it (distance 1)
//      and of the outer ring (distance 2; its four corners are read by no
//      stencil and are left out);
//   B  collision of the tile and of the collision ring: the eight moving
//      populations into LDS;
//   C  pull streaming and the entropy update of the tile, stored.
// Thread t owns tile nodes t, t + 256, ... (row-major, so a wave covers
// whole row segments and its loads and stores are coalesced) and ring
// nodes t, t + 256, ... of the ring list (collision ring first).  A node's
// own moments stay in its owner's registers from A to C; LDS holds only
// what neighbours read.  The per-node arithmetic is the row sweep's, in the
// same order, and neighbour indices go through map_index on both axes, so
// every boundary rule of the row sweep holds and a tile may reach past the
// domain's edge (nodes outside it are neither updated nor stored).
#pragma once

namespace hlbm {
namespace HLBM_NS {

constexpr int kTileThreads = 256;

template <int TW, int TH>
struct TileGeom {
  static constexpr int AW = TW + 4, AH = TH + 4, NA = AW * AH;  // moments: distance <= 2
  static constexpr int BW = TW + 2, BH = TH + 2, NB = BW * BH;  // collision: distance <= 1
  static constexpr int NI = TW * TH;                            // tile nodes
  static constexpr int NBR = 2 * (TW + 2) + 2 * TH;             // collision ring
  static constexpr int NAR = 2 * (TW + 2) + 2 * (TH + 2);       // outer ring, corners left out
  static constexpr int KI = NI / kTileThreads;                  // tile nodes per thread
  static constexpr int KR = (NBR + NAR + kTileThreads - 1) / kTileThreads;
  static_assert(NI % kTileThreads == 0, "tile nodes must be a multiple of the workgroup");
};

// LDS of one tile.  Moments arrays are indexed (y + 2) AW + (x + 2) in tile
// coordinates (x, y), populations (y + 1) BW + (x + 1).
template <int TW, int TH>
struct TileLDS {
  using G = TileGeom<TW, TH>;
  real ux[G::NA], uy[G::NA], gx[G::NA], gy[G::NA], s[G::NA], lap[G::NA];
  real f[8][G::NB];  // populations 1..8 after collision
};

// Ring node r in tile coordinates: the collision ring's rows y = -1 and
// y = TH (x = -1..TW), then its columns x = -1 and x = TW (y = 0..TH-1),
// then the outer ring's rows y = -2 and y = TH+1 (x = -1..TW) and columns
// x = -2 and x = TW+1 (y = -1..TH).
template <int TW, int TH>
__device__ __forceinline__ void ring_node(int r, int &x, int &y) {
  constexpr int W2 = TW + 2;
  constexpr int NBR = TileGeom<TW, TH>::NBR;
  if (r < NBR) {
    if (r < 2 * W2) {
      y = r < W2 ? -1 : TH;
      x = (r < W2 ? r : r - W2) - 1;
    } else {
      r -= 2 * W2;
      x = r < TH ? -1 : TW;
      y = r < TH ? r : r - TH;
    }
  } else {
    r -= NBR;
    if (r < 2 * W2) {
      y = r < W2 ? -2 : TH + 1;
      x = (r < W2 ? r : r - W2) - 1;
    } else {
      r -= 2 * W2;
      x = r < TH + 2 ? -2 : TW + 1;
      y = (r < TH + 2 ? r : r - (TH + 2)) - 1;
    }
  }
}

// Moments of one node kept by its owner from A to B and C.
struct TileNode {
  real dr, rho, pxx, pyy, pxy, ux, uy, th, sv;
};

// One tile (tx, ty) of one domain; returns once its loads are issued when
// any thread's `frozen` is nonzero (see domain_frozen).  The first barrier, after
// the loads are issued, also keeps the previous item's LDS reads ahead of
// this item's writes.
template <int TW, int TH>
__device__ __forceinline__ void tile_step(const DomainArgs &d, const real *src0, real *dst0,
                                          unsigned *status, const int tx, const int ty,
                                          const unsigned frozen, TileLDS<TW, TH> &L) {
  using G = TileGeom<TW, TH>;
  constexpr int K = G::KI + G::KR;
  constexpr unsigned kEl = sizeof(real);
  const int t = threadIdx.x;
  const int x0 = tx * TW, y0 = ty * TH;
  unsigned bad = 0;

  // ---------------- node of each slot: tile slots first, then ring slots
  int px[K], py[K];
  bool live[K];  // ring slots past the end of the ring list are idle
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (k < G::KI) {
      const int n = t + k * kTileThreads;
      py[k] = n / TW;
      px[k] = n - py[k] * TW;
      live[k] = true;
    } else {
      const int r = t + (k - G::KI) * kTileThreads;
      live[k] = r < G::NBR + G::NAR;
      ring_node<TW, TH>(live[k] ? r : 0, px[k], py[k]);
    }
  }

  // ---------------- A: issue every load, then the moments
  real ld[K][kPlanes];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (live[k]) {
      const int cx = map_index(x0 + px[k], d.nx, d.bcx);
      const int cy = map_index(y0 + py[k], d.ny, d.bcy);
      const unsigned off = (unsigned)(cy * d.pitch + cx) * kEl;
#pragma unroll
      for (int q = 0; q < kPlanes; ++q) ld[k][q] = load_at(src0 + (long long)q * d.plane, off);
    }
  }
  if (barrier_skip<true>(frozen)) return;
  TileNode own[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (!live[k]) continue;
    real F[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) F[q] = ld[k][q];
    const real sv = ld[k][9];
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
    const int ia = (py[k] + 2) * G::AW + (px[k] + 2);
    L.ux[ia] = ux;
    L.uy[ia] = uy;
    L.lap[ia] = lap_val;
    L.gx[ia] = m.rho * ux * ((real(1) - th) - ux * ux);
    L.gy[ia] = m.rho * uy * ((real(1) - th) - uy * uy);
    L.s[ia] = sv;
    own[k] = TileNode{m.dr, m.rho, m.pxx, m.pyy, m.pxy, ux, uy, th, sv};
    bad |= (m.rho > real(0) && th > real(0) && __builtin_isfinite(ux + uy + th)) ? 0u : 1u;
  }
  __syncthreads();

  // ---------------- B: collision of the tile and the collision ring
  const real cs2 = real(kCs2);
  const real cref = cs2 * (d.theta_ref - real(1));
  real keep_f0[G::KI], keep_phi[G::KI];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (k >= G::KI && t + (k - G::KI) * kTileThreads >= G::NBR) continue;
    const TileNode &o = own[k];
    const int i = (py[k] + 2) * G::AW + (px[k] + 2);
    const real rho = o.rho, ux = o.ux, uy = o.uy, th = o.th, dr = o.dr;
    const real uxe = L.ux[i + 1], uxw = L.ux[i - 1];
    const real uye = L.uy[i + 1], uyw = L.uy[i - 1];
    const real uxn = L.ux[i + G::AW], uxs = L.ux[i - G::AW];
    const real uyn = L.uy[i + G::AW], uys = L.uy[i - G::AW];
    const real dxux = real(0.5) * (uxe - uxw), dxuy = real(0.5) * (uye - uyw);
    const real dyux = real(0.5) * (uxn - uxs), dyuy = real(0.5) * (uyn - uys);
    const real div = dxux + dyuy;
    const real p = rho * cs2 * th;
    const real dth = th - d.theta_ref;
    const real dp = cs2 * (dr * th + d.rho_ref * dth);  // p - p_ref
    const real tau = div_fast(d.mu, p);
    const real taub = tau + real(0.5);
    const real itaub = rcp_fast(taub);
    const real gc = L.gx[i];
    const real gxe = L.gx[i + 1], gxw = L.gx[i - 1];
    const real gcy = L.gy[i];
    const real gyn = L.gy[i + G::AW], gys = L.gy[i - G::AW];
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
    const real prxx = (o.pxx - dp) - ruxx + real(0.5) * Exx;
    const real pryy = (o.pyy - dp) - ruyy + real(0.5) * Eyy;
    const real prxy = o.pxy - ruxy;
    const real tp = taub * p;
    const real fdxx = -tp * (dxux - dyuy);
    const real fdxy = -tp * (dyux + dxuy);
    // wall rows (by their unwrapped row index, as in the row sweep) take the
    // projected stress alone
    const int yk = y0 + py[k];
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
    const real drc = dp - cs2 * dr;
    const real dc = cs2 * dth;
    const real drc2 = dr * c * c + d.rho_ref * dc * (c + cref);
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
    project(dr, rux, ruy, Axx, Axy, Ayy, Axxy, Axyy, Axxyy, f);
    const int j = (py[k] + 1) * G::BW + (px[k] + 1);
#pragma unroll
    for (int q = 1; q < kQ; ++q) L.f[q - 1][j] = f[q];
    if (k < G::KI) {
      real phi;
      if (d.flags & kFlagPhiFD) {
        const real aa = dxux - dyuy, bb = dyux + dxuy;
        phi = d.mu * (aa * aa + bb * bb);
      } else {
        phi = -(tau * itaub) * (a1xx * dxux + a1xy * (dyux + dxuy) + a1yy * dyuy);
      }
      keep_f0[k < G::KI ? k : 0] = f[0];
      keep_phi[k < G::KI ? k : 0] = phi;
    }
  }
  __syncthreads();

  // ---------------- C: streaming and entropy of the tile's nodes
#pragma unroll
  for (int k = 0; k < G::KI; ++k) {
    const int x = x0 + px[k], y = y0 + py[k];
    if (x >= d.nx || y >= d.ny) continue;
    const TileNode &o = own[k];
    const int j = (py[k] + 1) * G::BW + (px[k] + 1);
    const int i = (py[k] + 2) * G::AW + (px[k] + 2);
    real Fo[kQ];
    Fo[0] = keep_f0[k];
    Fo[1] = L.f[0][j - 1];               // from x - 1
    Fo[3] = L.f[2][j + 1];               // from x + 1
    Fo[2] = L.f[1][j - G::BW];           // from y - 1
    Fo[5] = L.f[4][j - G::BW - 1];       // from (x - 1, y - 1)
    Fo[6] = L.f[5][j - G::BW + 1];       // from (x + 1, y - 1)
    Fo[4] = L.f[3][j + G::BW];           // from y + 1
    Fo[7] = L.f[6][j + G::BW + 1];       // from (x + 1, y + 1)
    Fo[8] = L.f[7][j + G::BW - 1];       // from (x - 1, y + 1)
    const real sc = o.sv;
    const real advx = muscl_term(o.ux, L.s[i - 2], L.s[i - 1], sc, L.s[i + 1], L.s[i + 2]);
    const real advy = muscl_term(o.uy, L.s[i - 2 * G::AW], L.s[i - G::AW], sc, L.s[i + G::AW],
                                 L.s[i + 2 * G::AW]);
    const real lap = ((L.lap[i + 1] + L.lap[i - 1]) + (L.lap[i + G::AW] + L.lap[i - G::AW])) -
                     real(4) * L.lap[i];
    const real snew = sc - (advx + advy) + div_fast(d.lambda * lap + keep_phi[k], o.rho * o.th);
    const unsigned off = (unsigned)(y * d.pitch + x) * kEl;
#pragma unroll
    for (int q = 0; q < kQ; ++q) store_stream(dst0 + (long long)q * d.plane, off, Fo[q]);
    store_stream(dst0 + 9LL * d.plane, off, snew);
  }
  if (bad) atomicOr(status, 1u);
}

// Persistent walk over (domain, tile x, tile y) items with the strip
// kernels' per-workgroup skip of frozen domains.
template <int TW, int TH>
__global__ __launch_bounds__(kTileThreads) void k_tile_batch(BatchArgs a) {
  __shared__ TileLDS<TW, TH> L;
  for (int it = blockIdx.x; it < a.nitems; it += gridDim.x) {
    const int4 w = a.items[it];
    const int dm = __builtin_amdgcn_readfirstlane(w.x);
    const DomainArgs d = a.doms[dm];
    const long long off = a.offs[dm];
    // after the loads it must not wait for (memory counters drain in order)
    const unsigned frozen = domain_frozen(a.status + dm);
    tile_step<TW, TH>(d, a.src_buf + off, a.dst_buf + off, a.status + dm,
                      __builtin_amdgcn_readfirstlane(w.y), __builtin_amdgcn_readfirstlane(w.z),
                      frozen, L);
  }
}

}  // namespace HLBM_NS
}  // namespace hlbm
