// Host-side launch interface between the C ABI (hlbm_api.hip) and the
// per-precision kernel translation units.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

namespace hlbm {

// Domain description in host precision; each translation unit converts it
// to its device argument struct.
struct HostDomain {
  long long plane;
  int nx, ny, pitch, bcx, bcy, flags;
  double mu, sigma, lambda, inv_cv, gm1, e2c, gamma, sgn_eps;
  double rho_ref, theta_ref, log_rho_ref, s_ref;
  double fref[9];
  double wall_u_lo, wall_u_hi, wall_theta;  // bcy == 2 (walls)
};

struct TileShape {
  int bw;        // tile width in columns (64, 128, 192 or 256); workgroup = bw + 64 lanes
  int rows;      // output rows per strip
  int xcd_remap; // 0 or 1
};

// Tile shape of the single-domain step for an nx x ny grid; tile_w, tile_h
// > 0 are taken as given.
//  - 192-column tiles with 16-row strips measured fastest at 8192^2 in FP32
//    (row segments stay 256-byte aligned, the halo wave is a quarter of the
//    workgroup, 16-row strips beat taller ones).  FP64 (elem_size 8), which
//    holds two workgroups per CU, runs 2-5 % faster with 32-row strips
//    there.  Grids narrower than 1024 columns keep 128-column tiles with
//    32-row strips (less ragged); from 1024 columns on, 192 x 8 measured
//    best or tied in FP32 (1024^2 37.0-37.6 k MLUPS against 35.4-37.3 k for
//    128 x 8, 1500^2 43.6 k against 39.1 k).
//  - Small grids get 64-column tiles (nx <= 64) and strips halved down to 4
//    rows until about 768 workgroups exist in FP32 (half a round of six per
//    CU; at 1024^2 192 x 8, 768 workgroups, edges out 192 x 4) and 512 in
//    FP64, whose sweep holds two workgroups per CU, so 512 fill the chip
//    once (at 1024^2 128 x 16 runs 15.8 k MLUPS against 13.4 k for
//    128 x 8): a strip is swept serially, so a few tall strips would leave
//    the chip idle.
inline TileShape step_tile(int nx, int ny, int tile_w, int tile_h, int elem_size) {
  TileShape t;
  t.bw = tile_w ? tile_w : (nx <= 64 ? 64 : (nx >= 1024 ? 192 : 128));
  int rows = tile_h ? tile_h : (t.bw == 192 && elem_size == 4 ? 16 : 32);
  if (!tile_h) {
    const long long nbx = (nx + t.bw - 1) / t.bw;
    const long long want = elem_size == 8 ? 512 : 768;
    while (rows > 4 && nbx * ((ny + rows - 1) / rows) < want) rows /= 2;
  }
  if (rows > ny) rows = ny;
  t.rows = rows;
  t.xcd_remap = 1;
  return t;
}

// Tile shape of the two-step sweep (periodic domains).  Its workgroup reads a
// radius-4 halo, rows + 8 rows for `rows` output rows, so it takes taller
// strips than the one-step sweep.  FP32 grids from 1024 columns on take
// 184-column tiles: tile plus halo fill three whole waves (192 columns leave
// a fourth wave with 8 of 64 lanes busy) and, with the s and theta rings cut
// to four rows, four workgroups fit a CU's LDS.  At 8192^2 (ms per step):
// 184 x 64 0.784, x 96 0.791, x 48 0.794, x 32 0.790 against 192 x 64 0.832
// (0.888 before the rings were cut).  Their strips are the tallest of 64,
// 32, 16 and 8 rows that give at least 768 workgroups and fill the last
// round of 1024 resident ones (four per CU on 256 CUs) at least three
// quarters: best or within 2 % of best at 1024^2 (8 rows), 1500^2 (16),
// 2048^2 (32), 3000^2 (64), 4096^2 (32), 6000^2 and 8192^2 (64), and
// 3-35 % faster than 192-column tiles from 1024^2 on, except level at
// 3000^2.  FP32 grids of 640 to 1023 columns take 120-column tiles (two
// whole waves, six workgroups per CU) with strips halved down to 8 rows
// until 768 workgroups exist: 8 rows at 768^2 and 1000^2, 29.3 and 41.3 k
// MLUPS against 25.0 and 30.9 k on 128-column tiles (at 512^2 the 128
// columns stay ahead, 13.8 against 13.1 k).  Narrower grids keep 128
// columns (halving the strips down to 8 rows until about 384 workgroups
// exist); FP64 keeps 128-column tiles, whose two levels of rings fit the
// LDS of one workgroup.
inline TileShape step2_tile(int nx, int ny, int tile_w, int tile_h, int elem_size) {
  TileShape t;
  const bool wide = nx >= 1024 && elem_size == 4;
  const bool mid = nx >= 640 && elem_size == 4;
  t.bw = tile_w ? tile_w : (nx <= 64 ? 64 : (wide ? 184 : (mid ? 120 : 128)));
  int rows = tile_h ? tile_h : 64;
  if (!tile_h) {
    const long long nbx = (nx + t.bw - 1) / t.bw;
    if (t.bw == 120) {
      while (rows > 8 && nbx * ((ny + rows - 1) / rows) < 768) rows /= 2;
    } else if (t.bw == 184) {
      constexpr long long kResident = 1024;
      for (; rows > 8; rows /= 2) {
        const long long nb = nbx * ((ny + rows - 1) / rows);
        const long long rounds = (nb + kResident - 1) / kResident;
        if (nb >= 768 && 4 * nb >= 3 * rounds * kResident) break;
      }
    } else {
      while (rows > 8 && nbx * ((ny + rows - 1) / rows) < 384) rows /= 2;
    }
  }
  if (rows > ny) rows = ny;
  t.rows = rows;
  t.xcd_remap = 1;
  return t;
}

// Elements from one state row to the next: nx rounded up to 64, so that every
// row, and with it every tile's row segment, starts 256-byte aligned (FP32).
// Rows of other widths lost 5 % (6000 and 14000 columns, rows 64-byte
// aligned) to 26 % (15446 columns, 24 bytes off a 64-byte boundary) of the
// step rate of their aligned neighbours.  The columns past nx are never read
// or written.
inline int row_pitch(int nx) { return (nx + 63) / 64 * 64; }

// Elements from one state plane to the next (elem_size 4 or 8): pitch x ny
// rounded up to 64.  A node's ten values sit at the same offset in every
// plane, and the step reads the same row segment from all ten at once.  With
// a plane size that is a multiple of a large power of two (8192^2 FP32: 256
// MiB) those ten segments land on the same HBM channels and banks.  Planes of
// 4 MiB or more therefore get a stride of a multiple of 128 KiB plus 64 KiB +
// 256 B (at most 0.2 MiB of padding per plane): 3 % faster at 8192^2 FP32
// than the bare 256 MiB stride, 1-2 % at 4096^2 and 6000^2.  Smaller planes
// keep a 64-element stride.
inline long long plane_stride(int nx, int ny, int elem_size) {
  const size_t es = (size_t)elem_size;
  const size_t elems = ((size_t)row_pitch(nx) * (size_t)ny + 63) / 64 * 64;
  if (elems * es < ((size_t)4 << 20)) return (long long)elems;
  const size_t unit = (size_t)128 << 10;
  const size_t bytes = (elems * es + unit - 1) / unit * unit + ((size_t)64 << 10) + 256;
  return (long long)(bytes / es);
}

// A pending learned correction for the tile kernels to apply as they load
// the state (x == nullptr: none): the moments and increments the
// correction kernels take, and the partial sums of correct_sums.
struct TileCorr {
  const float *x = nullptr, *dl = nullptr;
  const double *partials = nullptr;
  int conserve = 0;
};

#define HLBM_DECLARE_LAUNCHERS(NS)                                                          \
  namespace NS {                                                                            \
  hipError_t step(const HostDomain &d, const void *src, void *dst, unsigned *status,        \
                  const TileShape &tile, hipStream_t st);                                   \
  hipError_t step2(const HostDomain &d, const void *src, void *dst, unsigned *status,       \
                   const TileShape &tile, hipStream_t st);                                  \
  hipError_t init(const HostDomain &d, const void *rho, const void *ux, const void *uy,     \
                  const void *s, void *dst, hipStream_t st);                                \
  hipError_t wall(const HostDomain &d, void *state, hipStream_t st);                        \
  hipError_t moments(const HostDomain &d, const void *state, void *rho, void *ux, void *uy, \
                     void *s, void *theta, hipStream_t st);                                 \
  hipError_t populations(const HostDomain &d, void *state, void *F9, const void *s,         \
                         int to_state, hipStream_t st);                                     \
  hipError_t reduce(const HostDomain &d, const void *state, double *partials, int nparts,   \
                    double *out, hipStream_t st);                                           \
  hipError_t entropy(const void *rho, const void *theta, void *s, long long n, double gamma, \
                     hipStream_t st);                                                       \
  size_t domain_args_bytes();                                                               \
  void pack_domains(const HostDomain *h, int count, void *host_out);                        \
  hipError_t step_batch(const void *doms, const long long *offs, const void *items,          \
                        int nitems, const void *src, void *dst, unsigned *status, int rows, \
                        int cw, int grid, int xcd_walk, hipStream_t st);                    \
  int batch_blocks_per_cu(int cw);                                                          \
  hipError_t step_batch2(const void *doms, const long long *offs, const void *items,         \
                         int nitems, const void *src, void *dst, unsigned *status, int rows,\
                         int cw, int grid, int xcd_walk, hipStream_t st);                   \
  int batch2_blocks_per_cu(int cw);                                                         \
  hipError_t step_tile_batch(const void *doms, const long long *offs, const void *items,     \
                             int nitems, const void *src, void *dst, unsigned *status,       \
                             int tw, int th, int grid, int xcd_walk, void *mom,              \
                             const long long *foffs,                                         \
                             long long mom_sc, const TileCorr &corr, hipStream_t st);        \
  int tile_blocks_per_cu(int tw, int th);                                                   \
  bool tile_shape_supported(int tw, int th);                                                \
  hipError_t step_tile_batch2(const void *doms, const long long *offs, const void *items,    \
                              int nitems, const void *src, void *dst, unsigned *status,      \
                              int tw, int th, int grid, int xcd_walk, void *mom,             \
                              const long long *foffs,                                        \
                              long long mom_sc, const TileCorr &corr, hipStream_t st);       \
  int tile2_blocks_per_cu(int tw, int th);                                                  \
  bool tile2_shape_supported(int tw, int th);                                               \
  hipError_t correct(const void *doms, const long long *offs, int count, long long n,       \
                     void *state, const float *x, const float *dl, double *partials,        \
                     int conserve, hipStream_t st);                                         \
  size_t correct_partials_bytes(int count);                                                 \
  hipError_t correct_sums(const void *doms, const long long *offs, int count, long long n,  \
                          const float *x, const float *dl, double *partials, hipStream_t st); \
  hipError_t correct_apply(const void *doms, const long long *offs, int count, long long n, \
                           void *state, const float *x, const float *dl,                   \
                           const double *partials, int conserve, hipStream_t st);          \
  hipError_t batch_moments(const void *doms, const long long *offs, const long long *foffs, \
                           int count, long long maxn, const void *state, void *rho, void *ux,  \
                           void *uy, void *s, void *theta, hipStream_t st);                  \
  }

HLBM_DECLARE_LAUNCHERS(f32)
HLBM_DECLARE_LAUNCHERS(f64)

constexpr int kReduceParts = 1024;  // workgroups of the first reduction pass
constexpr int kReduceVals = 6;

}  // namespace hlbm
