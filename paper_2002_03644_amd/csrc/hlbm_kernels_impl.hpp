// Launchers of one precision; included by hlbm_kernels_f32.hip and
// hlbm_kernels_f64.hip after HLBM_REAL and HLBM_NS are defined.
#include "hlbm_device.hpp"
#include "closure_device.hpp"
#include "hlbm_launch.hpp"

namespace hlbm {
namespace HLBM_NS {

static DomainArgs to_device(const HostDomain &h) {
  DomainArgs d;
  d.plane = h.plane;
  d.nx = h.nx;
  d.pitch = h.pitch;
  d.ny = h.ny;
  d.bcx = h.bcx;
  d.bcy = h.bcy;
  d.flags = h.flags;
  d.mu = (real)h.mu;
  d.sigma = (real)h.sigma;
  d.lambda = (real)h.lambda;
  d.inv_cv = (real)h.inv_cv;
  d.gm1 = (real)h.gm1;
  d.e2c = (real)h.e2c;
  d.gamma = (real)h.gamma;
  d.sgn_eps = (real)h.sgn_eps;
  d.rho_ref = (real)h.rho_ref;
  d.theta_ref = (real)h.theta_ref;
  d.log_rho_ref = (real)h.log_rho_ref;
  d.s_ref = (real)h.s_ref;
  for (int q = 0; q < kQ; ++q) d.fref[q] = (real)h.fref[q];
  d.wall_u_lo = (real)h.wall_u_lo;
  d.wall_u_hi = (real)h.wall_u_hi;
  d.wall_theta = (real)h.wall_theta;
  return d;
}

static int grid_for(long long n, int threads) {
  long long b = (n + threads - 1) / threads;
  if (b > 65536) b = 65536;
  return (int)(b < 1 ? 1 : b);
}

hipError_t step(const HostDomain &h, const void *src, void *dst, unsigned *status,
                const TileShape &tile, hipStream_t st) {
  StepArgs a;
  a.d = to_device(h);
  a.src = (const real *)src;
  a.dst = (real *)dst;
  a.status = status;
  a.rows = tile.rows;
  a.nbx = (h.nx + tile.bw - 1) / tile.bw;
  a.nby = (h.ny + tile.rows - 1) / tile.rows;
  a.xcd_remap = tile.xcd_remap;
  const int nblk = a.nbx * a.nby;
  switch (tile.bw) {
  case 64:
    hipLaunchKernelGGL(k_step<64>, dim3(nblk), dim3(64 + 64), 0, st, a);
    break;
  case 128:
    hipLaunchKernelGGL(k_step<128>, dim3(nblk), dim3(128 + 64), 0, st, a);
    break;
  case 192:
    hipLaunchKernelGGL(k_step<192>, dim3(nblk), dim3(192 + 64), 0, st, a);
    break;
  case 256:
    hipLaunchKernelGGL(k_step<256>, dim3(nblk), dim3(256 + 64), 0, st, a);
    break;
  default:
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t step2(const HostDomain &h, const void *src, void *dst, unsigned *status,
                 const TileShape &tile, hipStream_t st) {
  StepArgs a;
  a.d = to_device(h);
  a.src = (const real *)src;
  a.dst = (real *)dst;
  a.status = status;
  a.rows = tile.rows;
  a.nbx = (h.nx + tile.bw - 1) / tile.bw;
  a.nby = (h.ny + tile.rows - 1) / tile.rows;
  a.xcd_remap = tile.xcd_remap;
  const dim3 grid(a.nbx * a.nby);
#define HLBM_STEP2_CASE(CW)                                                                  \
  case CW:                                                                                   \
    hipLaunchKernelGGL(k_step2<CW>, grid, dim3(step2_threads(CW)), 0, st, a);                \
    break;
  if (sizeof(real) == 4) {
    switch (tile.bw) {
      HLBM_STEP2_CASE(64)
      HLBM_STEP2_CASE(120)
      HLBM_STEP2_CASE(128)
      HLBM_STEP2_CASE(184)
      HLBM_STEP2_CASE(192)
      HLBM_STEP2_CASE(248)
      HLBM_STEP2_CASE(256)
    default:
      return hipErrorInvalidValue;
    }
  } else {
    switch (tile.bw) {
      HLBM_STEP2_CASE(64)
      HLBM_STEP2_CASE(128)
    default:
      return hipErrorInvalidValue;
    }
  }
#undef HLBM_STEP2_CASE
  return hipGetLastError();
}

hipError_t wall(const HostDomain &h, void *state, hipStream_t st) {
  WallArgs a;
  a.d = to_device(h);
  a.state = (real *)state;
  hipLaunchKernelGGL(k_wall, dim3(grid_for(2LL * h.nx, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t init(const HostDomain &h, const void *rho, const void *ux, const void *uy,
                const void *s, void *dst, hipStream_t st) {
  InitArgs a;
  a.d = to_device(h);
  a.rho = (const real *)rho;
  a.ux = (const real *)ux;
  a.uy = (const real *)uy;
  a.s = (const real *)s;
  a.dst = (real *)dst;
  const long long n = (long long)h.nx * h.ny;
  hipLaunchKernelGGL(k_init, dim3(grid_for(n, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t moments(const HostDomain &h, const void *state, void *rho, void *ux, void *uy,
                   void *s, void *theta, hipStream_t st) {
  FieldArgs a;
  a.d = to_device(h);
  a.state = (const real *)state;
  a.rho = (real *)rho;
  a.ux = (real *)ux;
  a.uy = (real *)uy;
  a.s = (real *)s;
  a.theta = (real *)theta;
  const long long n = (long long)h.nx * h.ny;
  hipLaunchKernelGGL(k_moments, dim3(grid_for(n, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t populations(const HostDomain &h, void *state, void *F9, const void *s, int to_state,
                       hipStream_t st) {
  PopArgs a;
  a.d = to_device(h);
  a.state = (real *)state;
  a.F9 = (real *)F9;
  a.s = (real *)s;
  a.to_state = to_state;
  const long long n = (long long)h.nx * h.ny;
  hipLaunchKernelGGL(k_populations, dim3(grid_for(n, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t reduce(const HostDomain &h, const void *state, double *partials, int nparts,
                  double *out, hipStream_t st) {
  ReduceArgs a;
  a.d = to_device(h);
  a.state = (const real *)state;
  a.partials = partials;
  hipLaunchKernelGGL(k_reduce, dim3(nparts), dim3(kRedThreads), 0, st, a);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, st, (const double *)partials,
                     nparts, out);
  return hipGetLastError();
}

hipError_t entropy(const void *rho, const void *theta, void *s, long long n, double gamma,
                   hipStream_t st) {
  const double cv = kCs2 / (gamma - 1.0);
  hipLaunchKernelGGL(k_entropy, dim3(grid_for(n, 256)), dim3(256), 0, st, (const real *)rho,
                     (const real *)theta, (real *)s, n, (real)(1.0 / cv), (real)(gamma - 1.0));
  return hipGetLastError();
}

size_t domain_args_bytes() { return sizeof(DomainArgs); }

void pack_domains(const HostDomain *h, int count, void *host_out) {
  DomainArgs *o = (DomainArgs *)host_out;
  for (int k = 0; k < count; ++k) o[k] = to_device(h[k]);
}

hipError_t step_batch(const void *doms, const long long *offs, const void *items, int nitems,
                      const void *src, void *dst, unsigned *status, int rows, int cw, int grid,
                      int xcd_walk, hipStream_t st) {
  BatchArgs a;
  a.xcd_walk = xcd_walk;
  a.doms = (const DomainArgs *)doms;
  a.offs = offs;
  a.items = (const int4 *)items;
  a.nitems = nitems;
  a.src_buf = (const real *)src;
  a.dst_buf = (real *)dst;
  a.status = status;
  a.rows = rows;
  a.mom = nullptr;
  a.foffs = nullptr;
  a.mom_sc = 0;
  a.cx = a.cdl = nullptr;
  a.cparts = nullptr;
  a.cconserve = 0;
  switch (cw) {
  case 64:
    hipLaunchKernelGGL(k_step_batch<64>, dim3(grid), dim3(64 + 64), 0, st, a);
    break;
  case 128:
    hipLaunchKernelGGL(k_step_batch<128>, dim3(grid), dim3(128 + 64), 0, st, a);
    break;
  case 120:  // odd last steps of batches on 120- and 184-column two-step strips (FP32)
    if (sizeof(real) != 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_step_batch<120>, dim3(grid), dim3(120 + 64), 0, st, a);
    break;
  case 184:
    if (sizeof(real) != 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_step_batch<184>, dim3(grid), dim3(184 + 64), 0, st, a);
    break;
  case 192:
    hipLaunchKernelGGL(k_step_batch<192>, dim3(grid), dim3(192 + 64), 0, st, a);
    break;
  case 256:
    hipLaunchKernelGGL(k_step_batch<256>, dim3(grid), dim3(256 + 64), 0, st, a);
    break;
  default:
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t step_batch2(const void *doms, const long long *offs, const void *items, int nitems,
                       const void *src, void *dst, unsigned *status, int rows, int cw, int grid,
                       int xcd_walk, hipStream_t st) {
  BatchArgs a;
  a.xcd_walk = xcd_walk;
  a.doms = (const DomainArgs *)doms;
  a.offs = offs;
  a.items = (const int4 *)items;
  a.nitems = nitems;
  a.src_buf = (const real *)src;
  a.dst_buf = (real *)dst;
  a.status = status;
  a.rows = rows;
  a.mom = nullptr;
  a.foffs = nullptr;
  a.mom_sc = 0;
  a.cx = a.cdl = nullptr;
  a.cparts = nullptr;
  a.cconserve = 0;
#define HLBM_BATCH2_CASE(CW)                                                                 \
  case CW:                                                                                   \
    hipLaunchKernelGGL(k_step_batch2<CW>, dim3(grid), dim3(step2_threads(CW)), 0, st, a);    \
    break;
  if (sizeof(real) == 4) {
    switch (cw) {
      HLBM_BATCH2_CASE(64)
      HLBM_BATCH2_CASE(120)
      HLBM_BATCH2_CASE(128)
      HLBM_BATCH2_CASE(184)
      HLBM_BATCH2_CASE(192)
    default:
      return hipErrorInvalidValue;
    }
  } else {
    switch (cw) {
      HLBM_BATCH2_CASE(64)
      HLBM_BATCH2_CASE(128)
    default:
      return hipErrorInvalidValue;
    }
  }
#undef HLBM_BATCH2_CASE
  return hipGetLastError();
}

int batch2_blocks_per_cu(int cw) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if (cw == 64)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch2<64>, step2_threads(64), 0);
  if (cw == 128)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch2<128>, step2_threads(128),
                                                     0);
  if (cw == 120 && sizeof(real) == 4)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch2<120>, step2_threads(120),
                                                     0);
  if (cw == 184 && sizeof(real) == 4)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch2<184>, step2_threads(184),
                                                     0);
  if (cw == 192 && sizeof(real) == 4)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch2<192>, step2_threads(192),
                                                     0);
  return e == hipSuccess && n > 0 ? n : 1;
}

// Shapes of the two-dimensional tile kernel (tile_w x tile_h, workgroup
// size) built for this precision; FP64 keeps the three whose registers and
// LDS leave at least two waves per SIMD.  The largest tiles take 512
// threads: fewer nodes per thread, half the registers, twice the waves.
#ifndef HLBM_TILE_SHAPES
#define HLBM_TILE_SHAPES(X) X(32, 8, 256) X(32, 16, 256) X(64, 8, 256) X(32, 32, 512) X(64, 16, 512)
#endif

// Shapes of the two-step tile kernel (FP32 only: its registers leave FP64
// one wave per SIMD).
#ifndef HLBM_TILE2_SHAPES
#define HLBM_TILE2_SHAPES(X) X(32, 16) X(64, 8)
#endif
constexpr int kTile2Threads = 512;  // workgroup of the two-step tile kernel

bool tile2_shape_supported(int tw, int th) {
#define HLBM_TILE_HAS(W, H) \
  if (tw == W && th == H) return true;
  HLBM_TILE2_SHAPES(HLBM_TILE_HAS)
#undef HLBM_TILE_HAS
  return false;
}

hipError_t step_tile_batch2(const void *doms, const long long *offs, const void *items,
                            int nitems, const void *src, void *dst, unsigned *status, int tw,
                            int th, int grid, int xcd_walk, void *mom, const long long *foffs,
                            long long mom_sc, const TileCorr &corr, hipStream_t st) {
  BatchArgs a;
  a.xcd_walk = xcd_walk;
  a.mom = (real *)mom;
  a.foffs = foffs;
  a.mom_sc = mom_sc;
  a.cx = corr.x;
  a.cdl = corr.dl;
  a.cparts = corr.partials;
  a.cconserve = corr.conserve;
  a.doms = (const DomainArgs *)doms;
  a.offs = offs;
  a.items = (const int4 *)items;
  a.nitems = nitems;
  a.src_buf = (const real *)src;
  a.dst_buf = (real *)dst;
  a.status = status;
  a.rows = th;
#define HLBM_TILE_CASE(W, H)                                                              \
  if (tw == W && th == H) {                                                               \
    if (a.cx)                                                                             \
      hipLaunchKernelGGL((k_tile_batch2<W, H, kTile2Threads, true>), dim3(grid),          \
                         dim3(kTile2Threads), 0, st, a);                                  \
    else                                                                                  \
      hipLaunchKernelGGL((k_tile_batch2<W, H, kTile2Threads, false>), dim3(grid),         \
                         dim3(kTile2Threads), 0, st, a);                                  \
    return hipGetLastError();                                                             \
  }
  HLBM_TILE2_SHAPES(HLBM_TILE_CASE)
#undef HLBM_TILE_CASE
  return hipErrorInvalidValue;
}

int tile2_blocks_per_cu(int tw, int th) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
#define HLBM_TILE_OCC(W, H)                                                                  \
  if (tw == W && th == H)                                                                    \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_tile_batch2<W, H, kTile2Threads,  \
                                                     false>, kTile2Threads, 0);
  HLBM_TILE2_SHAPES(HLBM_TILE_OCC)
#undef HLBM_TILE_OCC
  return e == hipSuccess && n > 0 ? n : 1;
}

bool tile_shape_supported(int tw, int th) {
#define HLBM_TILE_HAS(W, H, NT) \
  if (tw == W && th == H) return true;
  HLBM_TILE_SHAPES(HLBM_TILE_HAS)
#undef HLBM_TILE_HAS
  return false;
}

hipError_t step_tile_batch(const void *doms, const long long *offs, const void *items,
                           int nitems, const void *src, void *dst, unsigned *status, int tw,
                           int th, int grid, int xcd_walk, void *mom, const long long *foffs,
                           long long mom_sc, const TileCorr &corr, hipStream_t st) {
  BatchArgs a;
  a.xcd_walk = xcd_walk;
  a.mom = (real *)mom;
  a.foffs = foffs;
  a.mom_sc = mom_sc;
  a.cx = corr.x;
  a.cdl = corr.dl;
  a.cparts = corr.partials;
  a.cconserve = corr.conserve;
  a.doms = (const DomainArgs *)doms;
  a.offs = offs;
  a.items = (const int4 *)items;
  a.nitems = nitems;
  a.src_buf = (const real *)src;
  a.dst_buf = (real *)dst;
  a.status = status;
  a.rows = th;
#define HLBM_TILE_CASE(W, H, NT)                                                         \
  if (tw == W && th == H) {                                                              \
    if (a.cx)                                                                            \
      hipLaunchKernelGGL((k_tile_batch<W, H, NT, true>), dim3(grid), dim3(NT), 0, st, a); \
    else                                                                                 \
      hipLaunchKernelGGL((k_tile_batch<W, H, NT, false>), dim3(grid), dim3(NT), 0, st, a); \
    return hipGetLastError();                                                            \
  }
  HLBM_TILE_SHAPES(HLBM_TILE_CASE)
#undef HLBM_TILE_CASE
  return hipErrorInvalidValue;
}

int tile_blocks_per_cu(int tw, int th) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
#define HLBM_TILE_OCC(W, H, NT)                                                             \
  if (tw == W && th == H)                                                                   \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_tile_batch<W, H, NT, false>, NT, 0);
  HLBM_TILE_SHAPES(HLBM_TILE_OCC)
#undef HLBM_TILE_OCC
  return e == hipSuccess && n > 0 ? n : 1;
}

static CorrArgs corr_args(const void *doms, const long long *offs, int count, long long n,
                          void *state, const float *x, const float *dl, const double *partials,
                          int conserve) {
  CorrArgs a;
  a.doms = (const DomainArgs *)doms;
  a.offs = offs;
  a.state = (real *)state;
  a.x = x;
  a.dl = dl;
  a.n = n;
  a.sc = n * count;
  a.partials = (double *)partials;
  a.conserve = conserve;
  return a;
}

hipError_t correct_sums(const void *doms, const long long *offs, int count, long long n,
                        const float *x, const float *dl, double *partials, hipStream_t st) {
  const CorrArgs a = corr_args(doms, offs, count, n, nullptr, x, dl, partials, 1);
  hipLaunchKernelGGL(k_corr_sums, dim3(kCorrParts, count), dim3(kCorrThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t correct_apply(const void *doms, const long long *offs, int count, long long n,
                         void *state, const float *x, const float *dl, const double *partials,
                         int conserve, hipStream_t st) {
  const CorrArgs a = corr_args(doms, offs, count, n, state, x, dl, partials, conserve);
  const long long per = (n + kCorrThreads - 1) / kCorrThreads;
  const int gx = (int)(per < 256 ? per : 256);
  hipLaunchKernelGGL(k_corr_apply, dim3(gx, count), dim3(kCorrThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t correct(const void *doms, const long long *offs, int count, long long n, void *state,
                   const float *x, const float *dl, double *partials, int conserve,
                   hipStream_t st) {
  if (conserve) {
    const hipError_t e = correct_sums(doms, offs, count, n, x, dl, partials, st);
    if (e != hipSuccess) return e;
  }
  return correct_apply(doms, offs, count, n, state, x, dl, partials, conserve, st);
}

hipError_t batch_moments(const void *doms, const long long *offs, const long long *foffs,
                         int count, long long maxn, const void *state, void *rho, void *ux,
                         void *uy, void *s, void *theta, hipStream_t st) {
  BatchFieldArgs a;
  a.doms = (const DomainArgs *)doms;
  a.offs = offs;
  a.foffs = foffs;
  a.state = (const real *)state;
  a.rho = (real *)rho;
  a.ux = (real *)ux;
  a.uy = (real *)uy;
  a.s = (real *)s;
  a.theta = (real *)theta;
  const long long per = (maxn + 255) / 256;
  const int gx = (int)(per < 128 ? per : 128);
  hipLaunchKernelGGL(k_batch_moments, dim3(gx, count), dim3(256), 0, st, a);
  return hipGetLastError();
}

size_t correct_partials_bytes(int count) {
  return sizeof(double) * kCorrParts * kCorrVals * (size_t)count;
}

int batch_blocks_per_cu(int cw) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if (cw == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch<64>, 128, 0);
  if (cw == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch<128>, 192, 0);
  if (cw == 120 && sizeof(real) == 4)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch<120>, 184, 0);
  if (cw == 184 && sizeof(real) == 4)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch<184>, 248, 0);
  if (cw == 192) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch<192>, 256, 0);
  if (cw == 256) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch<256>, 320, 0);
  return e == hipSuccess && n > 0 ? n : 1;
}

}  // namespace HLBM_NS
}  // namespace hlbm
