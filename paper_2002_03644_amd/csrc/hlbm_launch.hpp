// Host-side launch interface between the C ABI (hlbm_api.cpp) and the
// per-precision kernel translation units.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

namespace hlbm {

// Domain description in host precision; each translation unit converts it
// to its device argument struct.
struct HostDomain {
  long long plane;
  int nx, ny, bcx, bcy, flags;
  double mu, sigma, lambda, inv_cv, gm1, e2c, gamma, sgn_eps;
  double rho_ref, theta_ref, log_rho_ref, s_ref;
  double fref[9];
  double wall_u_lo, wall_u_hi, wall_theta;  // bcy == 2 (walls)
};

struct TileShape {
  int bw;        // tile width in columns (64, 128 or 256); workgroup = bw + 64 lanes
  int rows;      // output rows per strip
  int xcd_remap; // 0 or 1
};

#define HLBM_DECLARE_LAUNCHERS(NS)                                                          \
  namespace NS {                                                                            \
  hipError_t step(const HostDomain &d, const void *src, void *dst, unsigned *status,        \
                  const TileShape &tile, hipStream_t st);                                   \
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
                        int cw, int grid, hipStream_t st);                                  \
  int batch_blocks_per_cu(int cw);                                                          \
  hipError_t correct(const void *doms, const long long *offs, int count, long long n,       \
                     void *state, const float *x, const float *dl, double *partials,        \
                     int conserve, hipStream_t st);                                         \
  size_t correct_partials_bytes(int count);                                                 \
  hipError_t batch_moments(const void *doms, const long long *offs, const long long *foffs, \
                           int count, long long maxn, const void *state, void *rho, void *ux,  \
                           void *uy, void *s, void *theta, hipStream_t st);                  \
  }

HLBM_DECLARE_LAUNCHERS(f32)
HLBM_DECLARE_LAUNCHERS(f64)

constexpr int kReduceParts = 1024;  // workgroups of the first reduction pass
constexpr int kReduceVals = 6;

}  // namespace hlbm
