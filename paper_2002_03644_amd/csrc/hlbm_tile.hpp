// Steps on two-dimensional tiles, for batches of small domains (included by
// hlbm_device.hpp after the row sweeps).
//
// The row sweeps pipeline a strip of rows through the stages; each strip
// reads rows + 4 input rows and pays a serial fill of the pipeline.  A 256^2
// domain cut into enough strips to fill the chip has strips of four rows:
// eight input rows for four output rows, and every wave runs every stage of
// every row, halo lanes included.  These kernels load a TW x TH tile and its
// halo at once and run the stages over the whole tile, with a barrier
// between them:
//   A  moments of the tile, of the collision ring around it (distance 1)
//      and of the outer ring (distance 2; its four corners are read by no
//      stencil and are left out);
//   B  collision of the tile and of the collision ring: the eight moving
//      populations into LDS;
//   C  pull streaming and the entropy update of the tile.
// Thread t of NT owns the slot nodes t, t + NT, ... of the list "tile nodes
// (row-major, so a wave covers whole row segments and its loads and stores
// are coalesced), collision ring, outer ring".  A node's own moments stay in
// its owner's registers from A to C; LDS holds only what neighbours read.
// The per-node arithmetic is the row sweep's, in the same order, and
// neighbour indices go through map_index on both axes, so every boundary
// rule of the row sweep holds and a tile may reach past the domain's edge
// (nodes outside it are neither updated nor stored).
//
// The two-step kernel (domains periodic on both axes, as for the two-step
// sweep) first runs the three stages on the virtual (TW + 4) x (TH + 4)
// tile around the output tile, which gives the intermediate state on the
// radius-2 halo the second step needs, hands that state over through LDS,
// and runs the stages again on the TW x TH tile: one load and one store of
// the state per two steps.  It runs 512 threads per workgroup: with 256 each
// thread holds twice the slots and 173 registers, two waves per SIMD, and
// 8 x 256^2 steps took 16.2 against 14.0 us (before the batch kernels'
// XCD-contiguous walk, which brought the 512-thread kernel to 13 us).
#pragma once

namespace hlbm {
namespace HLBM_NS {

constexpr int kTileThreads = 256;  // default workgroup of the tile kernels

template <int TW, int TH, int NT = kTileThreads>
struct TileGeom {
  static constexpr int AW = TW + 4, AH = TH + 4, NA = AW * AH;  // moments: distance <= 2
  static constexpr int BW = TW + 2, BH = TH + 2, NB = BW * BH;  // collision: distance <= 1
  static constexpr int NI = TW * TH;                            // tile nodes
  static constexpr int NBR = 2 * (TW + 2) + 2 * TH;             // collision ring
  static constexpr int NAR = 2 * (TW + 2) + 2 * (TH + 2);       // outer ring, corners left out
  static constexpr int NS = NI + NBR + NAR;                     // slot nodes
  static constexpr int K = (NS + NT - 1) / NT;                  // slots per thread
};

// LDS of one tile step.  Moments arrays are indexed (y + 2) AW + (x + 2) in
// tile coordinates (x, y), populations (y + 1) BW + (x + 1).
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

// The slots of one thread (item-independent) for NT threads.
template <int TW, int TH, int NT = kTileThreads>
struct TileSlots {
  static constexpr int K = TileGeom<TW, TH, NT>::K;
  int px[K], py[K];  // tile coordinates of each slot's node
  bool live[K];      // a node of the list (moments)
  bool coll[K];      // a tile or collision-ring node (collision)
  bool tile[K];      // a tile node (streaming and entropy)
};

template <int TW, int TH, int NT = kTileThreads>
__device__ __forceinline__ TileSlots<TW, TH, NT> tile_slots(const int t) {
  using G = TileGeom<TW, TH, NT>;
  TileSlots<TW, TH, NT> S;
#pragma unroll
  for (int k = 0; k < S.K; ++k) {
    const int g = t + k * NT;
    // slots wholly inside one part of the list fold to constants
    const bool all_tile = (k + 1) * NT <= G::NI;
    S.live[k] = (k + 1) * NT <= G::NS || g < G::NS;
    S.coll[k] = (k + 1) * NT <= G::NI + G::NBR || g < G::NI + G::NBR;
    S.tile[k] = all_tile || g < G::NI;
    if (all_tile || g < G::NI) {
      S.py[k] = g / TW;
      S.px[k] = g - S.py[k] * TW;
    } else {
      ring_node<TW, TH>(g < G::NS ? g - G::NI : 0, S.px[k], S.py[k]);
    }
  }
  return S;
}

// Moments of one node kept by its owner from A to B and C.
struct TileNode {
  real dr, rho, pxx, pyy, pxy, ux, uy, th, sv;
};

// Issue the ten loads of every live slot of the tile at (x0, y0).
template <int TW, int TH, int NT>
__device__ __forceinline__ void tile_loads(const DomainArgs &d, const real *src0, const int x0,
                                           const int y0, const TileSlots<TW, TH, NT> &S,
                                           real (&ld)[TileGeom<TW, TH, NT>::K][kPlanes]) {
  constexpr unsigned kEl = sizeof(real);
#pragma unroll
  for (int k = 0; k < S.K; ++k) {
    if (S.live[k]) {
      const int cx = map_index(x0 + S.px[k], d.nx, d.bcx);
      const int cy = map_index(y0 + S.py[k], d.ny, d.bcy);
      const unsigned off = (unsigned)(cy * d.pitch + cx) * kEl;
#pragma unroll
      for (int q = 0; q < kPlanes; ++q) ld[k][q] = load_at(src0 + (long long)q * d.plane, off);
    }
  }
}

// The pending correction (see BatchArgs) of every live slot's loaded state;
// dm: the domain, c: its conservation shifts.
template <int TW, int TH, int NT>
__device__ __forceinline__ void tile_correct(const DomainArgs &d, const BatchArgs &a, const int dm,
                                             const CorrShift &c, const int x0, const int y0,
                                             const TileSlots<TW, TH, NT> &S,
                                             real (&ld)[TileGeom<TW, TH, NT>::K][kPlanes]) {
  const long long fo = a.foffs[dm];
#pragma unroll
  for (int k = 0; k < S.K; ++k) {
    if (!S.live[k]) continue;
    const int cx = map_index(x0 + S.px[k], d.nx, d.bcx);
    const int cy = map_index(y0 + S.py[k], d.ny, d.bcy);
    const CorrDelta q = corr_delta(d, a.cx + fo, a.cdl + fo, a.mom_sc,
                                   (long long)cy * d.nx + cx, c);
#pragma unroll
    for (int p = 0; p < kQ; ++p) ld[k][p] += q.df[p];
    ld[k][9] = corr_s(ld[k][9], q);
  }
}

// A: moments of every live slot from its ten values into LDS and `own`.
template <int TW, int TH, int NT>
__device__ __forceinline__ void tile_a(const DomainArgs &d, const TileSlots<TW, TH, NT> &S,
                                       const real (&ld)[TileGeom<TW, TH, NT>::K][kPlanes],
                                       TileNode (&own)[TileGeom<TW, TH, NT>::K],
                                       TileLDS<TW, TH> &L, unsigned &bad) {
  using G = TileGeom<TW, TH>;
#pragma unroll
  for (int k = 0; k < S.K; ++k) {
    if (!S.live[k]) continue;
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
    const int ia = (S.py[k] + 2) * G::AW + (S.px[k] + 2);
    L.ux[ia] = ux;
    L.uy[ia] = uy;
    L.lap[ia] = lap_val;
    L.gx[ia] = m.rho * ux * ((real(1) - th) - ux * ux);
    L.gy[ia] = m.rho * uy * ((real(1) - th) - uy * uy);
    L.s[ia] = sv;
    own[k] = TileNode{m.dr, m.rho, m.pxx, m.pyy, m.pxy, ux, uy, th, sv};
    bad |= (m.rho > real(0) && th > real(0) && __builtin_isfinite(ux + uy + th)) ? 0u : 1u;
  }
}

// B: collision of the tile and the collision ring; the eight moving
// populations into LDS, population 0 and Phi into registers.  y0: the
// tile's row origin (wall rows go by the unwrapped row index, as in the row
// sweep).
template <int TW, int TH, int NT>
__device__ __forceinline__ void tile_b(const DomainArgs &d, const int y0,
                                       const TileSlots<TW, TH, NT> &S,
                                       const TileNode (&own)[TileGeom<TW, TH, NT>::K],
                                       TileLDS<TW, TH> &L, real (&keep_f0)[TileGeom<TW, TH, NT>::K],
                                       real (&keep_phi)[TileGeom<TW, TH, NT>::K]) {
  using G = TileGeom<TW, TH>;
  const real cs2 = real(kCs2);
  const real cref = cs2 * (d.theta_ref - real(1));
#pragma unroll
  for (int k = 0; k < S.K; ++k) {
    if (!S.coll[k]) continue;
    const TileNode &o = own[k];
    const int i = (S.py[k] + 2) * G::AW + (S.px[k] + 2);
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
    const int yk = y0 + S.py[k];
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
    const int j = (S.py[k] + 1) * G::BW + (S.px[k] + 1);
#pragma unroll
    for (int q = 1; q < kQ; ++q) L.f[q - 1][j] = f[q];
    real phi;
    if (d.flags & kFlagPhiFD) {
      const real aa = dxux - dyuy, bb = dyux + dxuy;
      phi = d.mu * (aa * aa + bb * bb);
    } else {
      phi = -(tau * itaub) * (a1xx * dxux + a1xy * (dyux + dxuy) + a1yy * dyuy);
    }
    keep_f0[k] = f[0];
    keep_phi[k] = phi;
  }
}

// C of slot k (a tile node): the streamed populations and the new entropy.
template <int TW, int TH, int NT>
__device__ __forceinline__ void tile_c(const DomainArgs &d, const int k,
                                       const TileSlots<TW, TH, NT> &S,
                                       const TileNode (&own)[TileGeom<TW, TH, NT>::K],
                                       const TileLDS<TW, TH> &L,
                                       const real (&keep_f0)[TileGeom<TW, TH, NT>::K],
                                       const real (&keep_phi)[TileGeom<TW, TH, NT>::K],
                                       real (&Fo)[kQ], real &snew) {
  using G = TileGeom<TW, TH>;
  const TileNode &o = own[k];
  const int j = (S.py[k] + 1) * G::BW + (S.px[k] + 1);
  const int i = (S.py[k] + 2) * G::AW + (S.px[k] + 2);
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
  snew = sc - (advx + advy) + div_fast(d.lambda * lap + keep_phi[k], o.rho * o.th);
}

// C of every tile slot, stored to the state at dst0 (tile origin x0, y0);
// with `mom` set also the moments of the new state (see BatchArgs), at
// mom + fo for this domain.
template <int TW, int TH, int NT>
__device__ __forceinline__ void tile_c_store(const DomainArgs &d, real *dst0, const int x0,
                                             const int y0, const TileSlots<TW, TH, NT> &S,
                                             const TileNode (&own)[TileGeom<TW, TH, NT>::K],
                                             const TileLDS<TW, TH> &L,
                                             const real (&keep_f0)[TileGeom<TW, TH, NT>::K],
                                             const real (&keep_phi)[TileGeom<TW, TH, NT>::K],
                                             real *mom, const long long mom_sc) {
  constexpr unsigned kEl = sizeof(real);
#pragma unroll
  for (int k = 0; k < S.K; ++k) {
    if (!S.tile[k]) continue;
    const int x = x0 + S.px[k], y = y0 + S.py[k];
    if (x >= d.nx || y >= d.ny) continue;
    real Fo[kQ], snew;
    tile_c<TW, TH>(d, k, S, own, L, keep_f0, keep_phi, Fo, snew);
    const unsigned off = (unsigned)(y * d.pitch + x) * kEl;
#pragma unroll
    for (int q = 0; q < kQ; ++q) store_stream(dst0 + (long long)q * d.plane, off, Fo[q]);
    store_stream(dst0 + 9LL * d.plane, off, snew);
    if (mom) {  // the arithmetic of k_batch_moments on the values just stored
      const NodeMoments m = node_moments(Fo, d);
      const long long i = (long long)y * d.nx + x;
      mom[i] = m.rho;
      mom[mom_sc + i] = m.jx / m.rho;
      mom[2 * mom_sc + i] = m.jy / m.rho;
      mom[3 * mom_sc + i] = node_theta(m.rho, snew, d);
    }
  }
}

// Persistent walk over (domain, tile x, tile y) items with the strip
// kernels' per-workgroup skip of frozen domains: one step per launch.
// kCorr: the variant that applies a pending correction (a.cx set), built
// apart so the plain steps do not carry its registers.
template <int TW, int TH, int NT, bool kCorr>
__global__ __launch_bounds__(NT) void k_tile_batch(BatchArgs a) {
  __shared__ TileLDS<TW, TH> L;
  __shared__ double ctot[kCorrVals];  // a pending correction's totals
  using G = TileGeom<TW, TH, NT>;
  const TileSlots<TW, TH, NT> S = tile_slots<TW, TH, NT>(threadIdx.x);
  const TileWalk walk = tile_walk(a.nitems, a.xcd_walk);
  for (int it = walk.first; it < walk.end; it += walk.step) {
    const int4 w = a.items[it];
    const int dm = __builtin_amdgcn_readfirstlane(w.x);
    const DomainArgs d = a.doms[dm];
    const long long off = a.offs[dm];
    // after the loads it must not wait for (memory counters drain in order)
    const unsigned frozen = domain_frozen(a.status + dm);
    const int x0 = __builtin_amdgcn_readfirstlane(w.y) * TW;
    const int y0 = __builtin_amdgcn_readfirstlane(w.z) * TH;
    real ld[G::K][kPlanes];
    tile_loads<TW, TH>(d, a.src_buf + off, x0, y0, S, ld);
    if (kCorr && a.cconserve && threadIdx.x < kCorrVals)
      ctot[threadIdx.x] = corr_total(a.cparts, dm, threadIdx.x);
    // one skip decision per workgroup; the barrier also keeps the previous
    // item's LDS reads ahead of this item's writes, and publishes ctot
    if (barrier_skip<true>(frozen)) continue;
    if constexpr (kCorr)
      tile_correct<TW, TH>(d, a, dm, corr_shift(ctot, (long long)d.nx * d.ny, a.cconserve), x0,
                           y0, S, ld);
    TileNode own[G::K];
    unsigned bad = 0;
    tile_a<TW, TH>(d, S, ld, own, L, bad);
    __syncthreads();
    real keep_f0[G::K], keep_phi[G::K];
    tile_b<TW, TH>(d, y0, S, own, L, keep_f0, keep_phi);
    __syncthreads();
    tile_c_store<TW, TH>(d, a.dst_buf + off, x0, y0, S, own, L, keep_f0, keep_phi,
                         a.mom ? a.mom + a.foffs[dm] : nullptr, a.mom_sc);
    if (bad) atomicOr(a.status + dm, 1u);
  }
}

// LDS of the two-step kernel: the first step's arrays, then the hand-over
// of its results (ten values per node of the virtual tile), then the second
// step's arrays, each region reused after a barrier.
template <int TW, int TH>
union TileLDS2 {
  TileLDS<TW + 4, TH + 4> l1;
  real xch[kPlanes][(TW + 4) * (TH + 4)];
  TileLDS<TW, TH> l2;
};

// Two steps per launch for domains periodic on both axes: step one on the
// virtual tile (TW + 4) x (TH + 4) at (x0 - 2, y0 - 2), whose results are
// exactly the intermediate state on the second step's tile and radius-2
// halo; step two on the TW x TH tile.
// Register budget: two workgroups of NT threads per compute unit (the
// correction variant would otherwise take more registers than that allows).
template <int TW, int TH, int NT, bool kCorr>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2 * NT / 256)))
void k_tile_batch2(BatchArgs a) {
  __shared__ TileLDS2<TW, TH> L;
  __shared__ double ctot[kCorrVals];  // a pending correction's totals
  using G1 = TileGeom<TW + 4, TH + 4, NT>;
  using G2 = TileGeom<TW, TH, NT>;
  constexpr int VW = TW + 4;  // row length of the hand-over
  const TileSlots<TW + 4, TH + 4, NT> S1 = tile_slots<TW + 4, TH + 4, NT>(threadIdx.x);
  const TileSlots<TW, TH, NT> S2 = tile_slots<TW, TH, NT>(threadIdx.x);
  const TileWalk walk = tile_walk(a.nitems, a.xcd_walk);
  for (int it = walk.first; it < walk.end; it += walk.step) {
    const int4 w = a.items[it];
    const int dm = __builtin_amdgcn_readfirstlane(w.x);
    const DomainArgs d = a.doms[dm];
    const long long off = a.offs[dm];
    const unsigned frozen = domain_frozen(a.status + dm);
    const int x0 = __builtin_amdgcn_readfirstlane(w.y) * TW;
    const int y0 = __builtin_amdgcn_readfirstlane(w.z) * TH;
    unsigned bad = 0;
    // ---------------- step one on the virtual tile
    real hand[G1::K][kPlanes];  // its results, by slot
    {
      real ld[G1::K][kPlanes];
      tile_loads<TW + 4, TH + 4>(d, a.src_buf + off, x0 - 2, y0 - 2, S1, ld);
      if (kCorr && a.cconserve && threadIdx.x < kCorrVals)
        ctot[threadIdx.x] = corr_total(a.cparts, dm, threadIdx.x);
      if (barrier_skip<true>(frozen)) continue;
      if constexpr (kCorr)
        tile_correct<TW + 4, TH + 4>(d, a, dm,
                                     corr_shift(ctot, (long long)d.nx * d.ny, a.cconserve),
                                     x0 - 2, y0 - 2, S1, ld);
      TileNode own[G1::K];
      tile_a<TW + 4, TH + 4>(d, S1, ld, own, L.l1, bad);
      __syncthreads();
      real keep_f0[G1::K], keep_phi[G1::K];
      tile_b<TW + 4, TH + 4>(d, y0 - 2, S1, own, L.l1, keep_f0, keep_phi);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < G1::K; ++k) {
        if (!S1.tile[k]) continue;
        real Fo[kQ], snew;
        tile_c<TW + 4, TH + 4>(d, k, S1, own, L.l1, keep_f0, keep_phi, Fo, snew);
#pragma unroll
        for (int q = 0; q < kQ; ++q) hand[k][q] = Fo[q];
        hand[k][9] = snew;
      }
    }
    __syncthreads();  // every read of the first step's arrays is done
#pragma unroll
    for (int k = 0; k < G1::K; ++k) {
      if (!S1.tile[k]) continue;
      const int v = S1.py[k] * VW + S1.px[k];
#pragma unroll
      for (int q = 0; q < kPlanes; ++q) L.xch[q][v] = hand[k][q];
    }
    __syncthreads();
    // ---------------- step two on the output tile
    real ld2[G2::K][kPlanes];
#pragma unroll
    for (int k = 0; k < G2::K; ++k) {
      if (!S2.live[k]) continue;
      const int v = (S2.py[k] + 2) * VW + (S2.px[k] + 2);
#pragma unroll
      for (int q = 0; q < kPlanes; ++q) ld2[k][q] = L.xch[q][v];
    }
    __syncthreads();  // the hand-over is read before the second step's arrays overwrite it
    TileNode own2[G2::K];
    tile_a<TW, TH>(d, S2, ld2, own2, L.l2, bad);
    __syncthreads();
    real keep2_f0[G2::K], keep2_phi[G2::K];
    tile_b<TW, TH>(d, y0, S2, own2, L.l2, keep2_f0, keep2_phi);
    __syncthreads();
    tile_c_store<TW, TH>(d, a.dst_buf + off, x0, y0, S2, own2, L.l2, keep2_f0, keep2_phi,
                         a.mom ? a.mom + a.foffs[dm] : nullptr, a.mom_sc);
    if (bad) atomicOr(a.status + dm, 1u);
  }
}

}  // namespace HLBM_NS
}  // namespace hlbm
