// C ABI of the hybrid LBM library (declared in include/hlbm.h): parameter
// validation, workspace layout, launches and status codes.  The workspace is
// the caller's device buffer; this file never allocates device memory.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include <hip/hip_runtime.h>

#include "hlbm.h"
#include "hlbm_launch.hpp"
#include "hlbm_nn.h"
#include "hlbm_nn_internal.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr double kCs2 = 1.0 / 3.0;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_size(int dtype) { return dtype == HLBM_F64 ? 8 : 4; }

long long plane_elems(const hlbm_params *p) {
  return hlbm::plane_stride(p->nx, p->ny, (int)elem_size(p->dtype));
}

struct Layout {
  size_t buffer;    // one ten-plane state buffer
  size_t off_buf1;  // second buffer
  size_t off_part;  // reduction partials
  size_t off_out;   // reduction result
  size_t off_stat;  // status word
  size_t total;
};

Layout layout_of(const hlbm_params *p) {
  Layout L;
  L.buffer = round_up((size_t)plane_elems(p) * 10 * elem_size(p->dtype), kAlign);
  L.off_buf1 = L.buffer;
  L.off_part = 2 * L.buffer;
  L.off_out = L.off_part + round_up(sizeof(double) * hlbm::kReduceParts * hlbm::kReduceVals, kAlign);
  L.off_stat = L.off_out + kAlign;
  L.total = L.off_stat + kAlign;
  return L;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

}  // namespace

struct hlbm_handle {
  hlbm_params p;
  hlbm::HostDomain dom;
  hlbm::TileShape tile;   // one step per launch
  hlbm::TileShape tile2;  // two steps per launch
  int spl;                // steps per launch (1 or 2)
  Layout L;
  char *ws;
  int cur;
  int64_t steps;
};

namespace {

char *buf(hlbm_handle *h, int which) { return h->ws + (which ? h->L.off_buf1 : 0); }
double *partials(hlbm_handle *h) { return (double *)(h->ws + h->L.off_part); }
double *red_out(hlbm_handle *h) { return (double *)(h->ws + h->L.off_out); }
unsigned *status_word(hlbm_handle *h) { return (unsigned *)(h->ws + h->L.off_stat); }

int hip_status(hipError_t e) { return e == hipSuccess ? HLBM_OK : HLBM_EHIP; }

// Reference populations f^eq_i(rho_ref, 0, theta_ref) of the FP32 deviation
// storage, from the nine Hermite coefficients of the rest equilibrium (the
// fourth-order one drops out when the expansion stops at third order).
void rest_equilibrium(double rho, double theta, int order, double f[9]) {
  const double c = kCs2 * (theta - 1.0);
  const double A0 = rho, Axx = rho * c, Ayy = rho * c, Axxyy = order == 3 ? 0.0 : rho * c * c;
  f[0] = 4.0 / 9.0 * (A0 - 1.5 * (Axx + Ayy) + 2.25 * Axxyy);
  const double bx = A0 + 3 * Axx - 1.5 * Ayy - 4.5 * Axxyy;
  f[1] = f[3] = bx / 9.0;
  const double by = A0 + 3 * Ayy - 1.5 * Axx - 4.5 * Axxyy;
  f[2] = f[4] = by / 9.0;
  const double bd = A0 + 3 * (Axx + Ayy) + 9 * Axxyy;
  f[5] = f[6] = f[7] = f[8] = bd / 36.0;
}

// Steps per launch of a batch domain: two-step sweeps need periodic axes
// (validated), and are the batch's choice for FP32 there (its two-step
// tiles serve small domains); FP64's two-level sweep holds one wave per SIMD.
int batch_steps_per_launch(const hlbm_params *p) {
  if (p->steps_per_launch) return p->steps_per_launch;
  const bool periodic = p->bc_x == HLBM_BC_PERIODIC && p->bc_y == HLBM_BC_PERIODIC;
  return periodic && p->dtype == HLBM_F32 ? 2 : 1;
}

// Steps per launch of a single domain: as for a batch domain, from
// kTwoStepMinNodes nodes on.  Smaller grids give the two-step sweep too few
// workgroups to fill the chip with its taller strips, and the one-step sweep
// is faster there (MLUPS, one against two steps per launch: 512^2 17.8 k /
// 13.5 k, 640^2 23.9 / 19.7, 768^2 28.0 / 27.7; 1000^2 35.8 / 38.4, 1024^2
// 37.3 / 39.9).
constexpr long long kTwoStepMinNodes = 900000;
int steps_per_launch(const hlbm_params *p) {
  if (p->steps_per_launch) return p->steps_per_launch;
  const int spl = batch_steps_per_launch(p);
  return spl == 2 && (long long)p->nx * p->ny < kTwoStepMinNodes ? 1 : spl;
}

hlbm::TileShape default_tile(const hlbm_params *p) {
  if (steps_per_launch(p) == 2)  // tile_w / tile_h belong to the two-step sweep
    return hlbm::step_tile(p->nx, p->ny, 0, 0, (int)elem_size(p->dtype));
  return hlbm::step_tile(p->nx, p->ny, p->tile_w, p->tile_h, (int)elem_size(p->dtype));
}

hlbm::TileShape default_tile2(const hlbm_params *p) {
  return hlbm::step2_tile(p->nx, p->ny, p->tile_w, p->tile_h, (int)elem_size(p->dtype));
}

void fill_domain(const hlbm_params *p, hlbm::HostDomain *d) {
  memset(d, 0, sizeof(*d));
  d->plane = plane_elems(p);
  d->nx = p->nx;
  d->pitch = hlbm::row_pitch(p->nx);
  d->ny = p->ny;
  d->bcx = p->bc_x;
  d->bcy = p->bc_y;
  d->flags = (p->phi_mode == HLBM_PHI_FD ? 1 : 0) | (p->e1_centred ? 2 : 0) | (p->e2_off ? 4 : 0) |
             (p->precise_theta ? 8 : 0) | (p->feq_order == 3 ? 16 : 0);
  const double g = p->gamma;
  const double cv = kCs2 / (g - 1.0), cp = g * kCs2 / (g - 1.0);
  d->mu = p->mu;
  d->sigma = p->sigma;
  d->sgn_eps = p->sgn_eps;
  d->lambda = p->mu * cp / p->prandtl;
  d->inv_cv = 1.0 / cv;
  d->gm1 = g - 1.0;
  d->e2c = (2.0 + 2.0) / 2.0 - g;  // (D + 2) / D - gamma with D = 2
  d->gamma = g;
  d->wall_u_lo = p->wall_ux_lo;
  d->wall_u_hi = p->wall_ux_hi;
  d->wall_theta = p->wall_theta;
  if (p->dtype == HLBM_F32) {
    d->rho_ref = p->rho_ref;
    d->theta_ref = p->theta_ref;
    d->log_rho_ref = log(p->rho_ref);
    d->s_ref = cv * log(p->theta_ref / pow(p->rho_ref, g - 1.0));
    rest_equilibrium(p->rho_ref, p->theta_ref, p->feq_order, d->fref);
  } else {
    d->rho_ref = 0.0;      // absolute populations
    d->theta_ref = 1.0;    // theta = exp(s / c_v + (gamma - 1) ln rho)
    d->log_rho_ref = 0.0;
    d->s_ref = 0.0;
  }
}

__global__ void k_clear_words(unsigned *w, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = 0u;
}

// Wall rows of a state buffer (nothing without walls).
hipError_t apply_walls(hlbm_handle *h, void *state, hipStream_t st) {
  if (h->p.bc_y != HLBM_BC_WALL) return hipSuccess;
  return h->p.dtype == HLBM_F64 ? hlbm::f64::wall(h->dom, state, st)
                                : hlbm::f32::wall(h->dom, state, st);
}

hipError_t run_reduce(hlbm_handle *h, double host[hlbm::kReduceVals], hipStream_t st) {
  hipError_t e;
  const void *state = buf(h, h->cur);
  if (h->p.dtype == HLBM_F64)
    e = hlbm::f64::reduce(h->dom, state, partials(h), hlbm::kReduceParts, red_out(h), st);
  else
    e = hlbm::f32::reduce(h->dom, state, partials(h), hlbm::kReduceParts, red_out(h), st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(host, red_out(h), sizeof(double) * hlbm::kReduceVals, hipMemcpyDeviceToHost,
                     st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

}  // namespace

extern "C" {

int hlbm_validate(const hlbm_params *p) {
  if (!p) return HLBM_EINVAL;
  if (p->nx < 1 || p->ny < 1) return HLBM_EINVAL;
  if ((long long)p->nx * (long long)p->ny * 9LL >= (1LL << 31)) return HLBM_EINVAL;
  if (p->dtype != HLBM_F64 && p->dtype != HLBM_F32) return HLBM_EINVAL;
  {
    // the step addresses a plane with (y pitch + x) in int and its byte
    // offset in 32 bits; padded rows make that larger than nx ny
    const long long rowel = (long long)hlbm::row_pitch(p->nx) * (long long)p->ny;
    if (rowel >= (1LL << 31)) return HLBM_EINVAL;
    if (rowel * (long long)elem_size(p->dtype) >= (1LL << 32)) return HLBM_EINVAL;
  }
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 2) return HLBM_EINVAL;
  if (p->bc_y == HLBM_BC_WALL &&
      (p->ny < 4 || !finite_pos(p->wall_theta) || !isfinite(p->wall_ux_lo) ||
       !isfinite(p->wall_ux_hi)))
    return HLBM_EINVAL;
  if (p->phi_mode != HLBM_PHI_LBM && p->phi_mode != HLBM_PHI_FD) return HLBM_EINVAL;
  if (p->e1_centred < 0 || p->e1_centred > 1 || p->e2_off < 0 || p->e2_off > 1) return HLBM_EINVAL;
  if (p->precise_theta < 0 || p->precise_theta > 1) return HLBM_EINVAL;
  if (p->feq_order != 0 && p->feq_order != 3 && p->feq_order != 4) return HLBM_EINVAL;
  if (p->steps_per_launch < 0 || p->steps_per_launch > 2) return HLBM_EINVAL;
  if (p->steps_per_launch == 2 &&
      (p->bc_x != HLBM_BC_PERIODIC || p->bc_y != HLBM_BC_PERIODIC ||
       (p->dtype == HLBM_F64 && p->tile_w != 0 && p->tile_w > 128)))
    return HLBM_EINVAL;
  if (p->tile_w != 0 && p->tile_w != 64 && p->tile_w != 128 && p->tile_w != 192 &&
      p->tile_w != 256 &&
      !((p->tile_w == 120 || p->tile_w == 184 || p->tile_w == 248) &&
        p->steps_per_launch == 2 && p->dtype == HLBM_F32))
    return HLBM_EINVAL;  // 120, 184 and 248: the two-step sweep's whole-wave widths
  if (p->tile_h < 0) return HLBM_EINVAL;
  if (!(isfinite(p->gamma) && p->gamma > 1.0)) return HLBM_EINVAL;
  if (!finite_pos(p->prandtl)) return HLBM_EINVAL;
  if (!(isfinite(p->mu) && p->mu >= 0.0)) return HLBM_EINVAL;
  if (!(isfinite(p->sigma) && p->sigma >= 0.0 && p->sigma <= 1.0)) return HLBM_EINVAL;
  if (!(isfinite(p->sgn_eps) && p->sgn_eps >= 0.0)) return HLBM_EINVAL;
  if (p->dtype == HLBM_F32 && !(finite_pos(p->rho_ref) && finite_pos(p->theta_ref)))
    return HLBM_EINVAL;
  return HLBM_OK;
}

int hlbm_launch_shape(const hlbm_params *p, int32_t *host_tile_w, int32_t *host_tile_h) {
  if (!host_tile_w || !host_tile_h || hlbm_validate(p) != HLBM_OK) return HLBM_EINVAL;
  const hlbm::TileShape t = steps_per_launch(p) == 2 ? default_tile2(p) : default_tile(p);
  *host_tile_w = t.bw;
  *host_tile_h = t.rows;
  return HLBM_OK;
}

int hlbm_launch_plan(const hlbm_params *p, int32_t *host_steps_per_launch, int32_t *host_tile_w,
                     int32_t *host_tile_h) {
  if (!host_steps_per_launch || !host_tile_w || !host_tile_h || hlbm_validate(p) != HLBM_OK)
    return HLBM_EINVAL;
  const int spl = steps_per_launch(p);
  const hlbm::TileShape t = spl == 2 ? default_tile2(p) : default_tile(p);
  *host_steps_per_launch = spl;
  *host_tile_w = t.bw;
  *host_tile_h = t.rows;
  return HLBM_OK;
}

size_t hlbm_workspace_bytes(const hlbm_params *p) {
  if (hlbm_validate(p) != HLBM_OK) return 0;
  return layout_of(p).total;
}

size_t hlbm_state_bytes(const hlbm_params *p) {
  if (hlbm_validate(p) != HLBM_OK) return 0;
  return (size_t)plane_elems(p) * 10 * elem_size(p->dtype);
}

int hlbm_init(hlbm_handle **out, const hlbm_params *p, void *workspace, size_t ws_bytes,
              const void *rho, const void *ux, const void *uy, const void *s,
              hlbm_stream_t stream) {
  if (!out) return HLBM_EINVAL;
  *out = nullptr;
  int v = hlbm_validate(p);
  if (v != HLBM_OK) return v;
  if (!rho || !ux || !uy || !s) return HLBM_EINVAL;
  const Layout L = layout_of(p);
  if (!workspace || ws_bytes < L.total) return HLBM_EWORKSPACE;
  if ((uintptr_t)workspace % kAlign != 0) return HLBM_EWORKSPACE;
  hlbm_handle *h = (hlbm_handle *)calloc(1, sizeof(hlbm_handle));
  if (!h) return HLBM_ENOMEM;
  h->p = *p;
  h->L = L;
  h->ws = (char *)workspace;
  h->cur = 0;
  h->steps = 0;
  h->tile = default_tile(p);
  h->tile2 = default_tile2(p);
  h->spl = steps_per_launch(p);
  fill_domain(p, &h->dom);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (p->dtype == HLBM_F64)
    e = hlbm::f64::init(h->dom, rho, ux, uy, s, buf(h, 0), st);
  else
    e = hlbm::f32::init(h->dom, rho, ux, uy, s, buf(h, 0), st);
  if (e == hipSuccess) e = apply_walls(h, buf(h, 0), st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, st, status_word(h), 64);
    e = hipGetLastError();
  }
  double host[hlbm::kReduceVals];
  if (e == hipSuccess) e = run_reduce(h, host, st);
  if (e != hipSuccess) {
    free(h);
    return HLBM_EHIP;
  }
  if (host[4] != 0.0) {  // non-finite, rho <= 0 or theta <= 0 in the input
    free(h);
    return HLBM_EINVAL;
  }
  *out = h;
  return host[5] >= 1.0 ? HLBM_WARN_CFL : HLBM_OK;
}

int hlbm_step(hlbm_handle *h, int32_t nsteps, hlbm_stream_t stream) {
  if (!h || nsteps < 0) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int32_t n = 0;
  if (h->spl == 2) {  // periodic domains, no walls
    for (; n + 2 <= nsteps; n += 2) {
      hipError_t e =
          h->p.dtype == HLBM_F64
              ? hlbm::f64::step2(h->dom, buf(h, h->cur), buf(h, h->cur ^ 1), status_word(h),
                                 h->tile2, st)
              : hlbm::f32::step2(h->dom, buf(h, h->cur), buf(h, h->cur ^ 1), status_word(h),
                                 h->tile2, st);
      if (e != hipSuccess) return HLBM_EHIP;
      h->cur ^= 1;
      h->steps += 2;
    }
  }
  for (; n < nsteps; ++n) {
    hipError_t e;
    if (h->p.dtype == HLBM_F64)
      e = hlbm::f64::step(h->dom, buf(h, h->cur), buf(h, h->cur ^ 1), status_word(h), h->tile, st);
    else
      e = hlbm::f32::step(h->dom, buf(h, h->cur), buf(h, h->cur ^ 1), status_word(h), h->tile, st);
    if (e == hipSuccess) e = apply_walls(h, buf(h, h->cur ^ 1), st);
    if (e != hipSuccess) return HLBM_EHIP;
    h->cur ^= 1;
    h->steps++;
  }
  return HLBM_OK;
}

int hlbm_moments(hlbm_handle *h, void *rho, void *ux, void *uy, void *s, void *theta,
                 hlbm_stream_t stream) {
  if (!h) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = h->p.dtype == HLBM_F64
                     ? hlbm::f64::moments(h->dom, buf(h, h->cur), rho, ux, uy, s, theta, st)
                     : hlbm::f32::moments(h->dom, buf(h, h->cur), rho, ux, uy, s, theta, st);
  return hip_status(e);
}

int hlbm_populations(hlbm_handle *h, void *F9, hlbm_stream_t stream) {
  if (!h || !F9) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = h->p.dtype == HLBM_F64
                     ? hlbm::f64::populations(h->dom, buf(h, h->cur), F9, nullptr, 0, st)
                     : hlbm::f32::populations(h->dom, buf(h, h->cur), F9, nullptr, 0, st);
  return hip_status(e);
}

int hlbm_set_populations(hlbm_handle *h, const void *F9, const void *s, hlbm_stream_t stream) {
  if (!h || !F9 || !s) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e =
      h->p.dtype == HLBM_F64
          ? hlbm::f64::populations(h->dom, buf(h, h->cur), (void *)F9, s, 1, st)
          : hlbm::f32::populations(h->dom, buf(h, h->cur), (void *)F9, s, 1, st);
  return hip_status(e);
}

int hlbm_totals(hlbm_handle *h, double *host_out4, hlbm_stream_t stream) {
  if (!h || !host_out4) return HLBM_EINVAL;
  double host[hlbm::kReduceVals];
  if (run_reduce(h, host, (hipStream_t)stream) != hipSuccess) return HLBM_EHIP;
  for (int k = 0; k < 4; ++k) host_out4[k] = host[k];
  return HLBM_OK;
}

int hlbm_status(hlbm_handle *h, double *host_max_cfl, hlbm_stream_t stream) {
  if (!h) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  double host[hlbm::kReduceVals];
  if (run_reduce(h, host, st) != hipSuccess) return HLBM_EHIP;
  unsigned word = 0;
  if (hipMemcpyAsync(&word, status_word(h), sizeof(unsigned), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return HLBM_EHIP;
  if (host_max_cfl) *host_max_cfl = host[5];
  return (host[4] != 0.0 || word != 0u) ? HLBM_EDIVERGED : HLBM_OK;
}

int hlbm_save_state(hlbm_handle *h, void *dst, hlbm_stream_t stream) {
  if (!h || !dst) return HLBM_EINVAL;
  const size_t bytes = hlbm_state_bytes(&h->p);
  return hip_status(hipMemcpyAsync(dst, buf(h, h->cur), bytes, hipMemcpyDeviceToDevice,
                                   (hipStream_t)stream));
}

int hlbm_load_state(hlbm_handle *h, const void *src, hlbm_stream_t stream) {
  if (!h || !src) return HLBM_EINVAL;
  const size_t bytes = hlbm_state_bytes(&h->p);
  return hip_status(hipMemcpyAsync(buf(h, h->cur), src, bytes, hipMemcpyDeviceToDevice,
                                   (hipStream_t)stream));
}

int64_t hlbm_steps_done(const hlbm_handle *h) { return h ? h->steps : -1; }

void hlbm_destroy(hlbm_handle *h) { free(h); }

const char *hlbm_strerror(int code) {
  switch (code) {
  case HLBM_OK: return "ok";
  case HLBM_WARN_CFL: return "initialised; the largest local CFL number is >= 1";
  case HLBM_EINVAL: return "invalid parameter, size, pointer or input field";
  case HLBM_EWORKSPACE: return "workspace missing, misaligned or too small";
  case HLBM_EHIP: return "HIP runtime call or kernel launch failed";
  case HLBM_EDIVERGED: return "state diverged (non-finite value, rho <= 0 or theta <= 0)";
  case HLBM_ENOMEM: return "host allocation failed";
  default: return "unknown status code";
  }
}

int hlbm_entropy_from_theta(int32_t dtype, double gamma, const void *rho, const void *theta,
                            void *s, int64_t n, hlbm_stream_t stream) {
  if (!rho || !theta || !s || n < 0 || !(gamma > 1.0)) return HLBM_EINVAL;
  if (dtype != HLBM_F64 && dtype != HLBM_F32) return HLBM_EINVAL;
  if (n == 0) return HLBM_OK;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = dtype == HLBM_F64 ? hlbm::f64::entropy(rho, theta, s, n, gamma, st)
                                   : hlbm::f32::entropy(rho, theta, s, n, gamma, st);
  return hip_status(e);
}

}  // extern "C"

// ======================================================================
// Totals of a raw state buffer with library-owned scratch (no allocation)
// ======================================================================
// Reduction partials and result of hlbm_state_totals: a fixed-size array in
// device memory, one copy per GPU, held until the process ends.  In host
// code this name is only a handle for hipGetSymbolAddress; kernels receive
// the device address that call returns.
constexpr int kScratchDoubles = hlbm::kReduceParts * hlbm::kReduceVals + 32;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double *scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current); nullptr if the lookup fails.
double *device_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    scratch_ptr[dev] = (double *)ptr;
  }
  return scratch_ptr[dev];
}

}  // namespace

extern "C" {

int hlbm_state_totals(const hlbm_params *p, const void *state, double *host_out4,
                      hlbm_stream_t stream) {
  if (hlbm_validate(p) != HLBM_OK || !state || !host_out4) return HLBM_EINVAL;
  double *ws = device_scratch();
  if (!ws) return HLBM_EHIP;
  hlbm::HostDomain dom;
  fill_domain(p, &dom);
  hipStream_t st = (hipStream_t)stream;
  double *parts = ws;
  double *out = ws + hlbm::kReduceParts * hlbm::kReduceVals;
  hipError_t e = p->dtype == HLBM_F64
                     ? hlbm::f64::reduce(dom, state, parts, hlbm::kReduceParts, out, st)
                     : hlbm::f32::reduce(dom, state, parts, hlbm::kReduceParts, out, st);
  double host[hlbm::kReduceVals];
  if (e == hipSuccess)
    e = hipMemcpyAsync(host, out, sizeof(double) * hlbm::kReduceVals, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return HLBM_EHIP;
  for (int k = 0; k < 4; ++k) host_out4[k] = host[k];
  return HLBM_OK;
}

}  // extern "C"

// ======================================================================
// Batched domains
// ======================================================================

struct hlbm_batch {
  int count = 0, dtype = 0;
  std::vector<hlbm_params> params;
  std::vector<hlbm::HostDomain> doms;
  std::vector<long long> offs;        // element offset of each domain's state in a buffer
  std::vector<long long> field_offs;  // offset of each domain in the concatenated fields
  std::vector<long long> state_elems; // ten planes of each domain
  char *ws = nullptr;
  size_t off_buf1 = 0, off_doms = 0, off_offs = 0, off_foffs = 0, off_items = 0, off_stat = 0;
  size_t off_corr = 0;
  size_t total = 0;
  size_t state_bytes = 0;             // one buffer
  int max_items = 0, nitems = 0, tile_w = 128, tile_h = 32, grid = 1, cur = 0, ncu = 1;
  int kind = HLBM_BATCH_STRIPS;  // kernel: row strips or two-dimensional tiles
  int spl = 1;         // steps per launch of the current kernel
  int spl_strips = 1;  // steps per launch of the strip kernel (2: every domain periodic, FP32)
  int grid1 = 1;  // persistent grid of the one-step kernel (odd last steps)
  int64_t steps = 0, nodes = 0;
  // captured plain steps: graph[0] one ping-pong pair, graph[1] kLongPairs
  // pairs (fewer replays, so fewer gaps between them, for short steps)
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int graph_cur[2] = {-1, -1};
  // captured corrected cycles (hlbm_closure_step): cgraph[0] two cycles,
  // cgraph[1] kLongCycles, each with the key it was captured under
  hipGraphExec_t cgraph[2] = {nullptr, nullptr};
  struct ClosureKey {
    int cur = -1, conserve = -1, version = -1, every = -1;
    int pending = -1;  // whether the captured cycles start with a pending correction
    const hlbm_cnn *net = nullptr;
    bool operator==(const ClosureKey &o) const {
      return cur == o.cur && conserve == o.conserve && version == o.version &&
             every == o.every && pending == o.pending && net == o.net;
    }
  } cgraph_key[2];
  int xcd_walk = 0;  // batch kernels: each XCD walks a contiguous range of the items
};

namespace {

// strip widths; 120 and 184 (tile plus halo in two and three whole waves)
// for two-step strips only, FP32
constexpr int kBatchTileW[6] = {64, 120, 128, 184, 192, 256};
constexpr int kBatchMinRows = 4;  // short strips: small domains are bound by the serial sweep
// Batches whose two state buffers fit in this many bytes (the 256 MiB
// last-level cache) walk their items XCD by XCD, which keeps neighbouring
// tiles' halos in one L2: 8 x 256^2 two-step tiles 14.3 -> 13.2 us per step,
// one-step 32 x 16 tiles 18.8 -> 15.0, 8 x 128^2 7.6 -> 5.8.  Larger batches
// stream from HBM, where the round-robin walk measured faster (8 x 1024^2
// strips 117.5 against 133 us per step).
constexpr size_t kXcdWalkBytes = (size_t)256 << 20;
// shapes of the two-dimensional tile kernel, tried in this order by the autotuner
constexpr int kTileShapes[5][2] = {{32, 8}, {32, 16}, {64, 8}, {32, 32}, {64, 16}};

int batch_items_for(const hlbm_batch *b, int tw, int th, std::vector<int> *out) {
  // largest domains first: every workgroup's walk then ends on small items
  std::vector<int> order(b->count);
  for (int k = 0; k < b->count; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (long long)b->params[x].nx * b->params[x].ny >
           (long long)b->params[y].nx * b->params[y].ny;
  });
  int n = 0;
  for (int k : order) {
    const int rows = std::min(th, b->params[k].ny);
    const int nbx = (b->params[k].nx + tw - 1) / tw, nby = (b->params[k].ny + rows - 1) / rows;
    for (int by = 0; by < nby; ++by)
      for (int bx = 0; bx < nbx; ++bx) {
        if (out) {
          out->push_back(k);
          out->push_back(bx);
          out->push_back(by);
          out->push_back(rows);
        }
        ++n;
      }
  }
  return n;
}

void batch_layout(hlbm_batch *b) {
  const size_t el = elem_size(b->dtype);
  long long acc = 0;
  b->offs.resize(b->count);
  b->state_elems.resize(b->count);
  b->field_offs.resize(b->count);
  long long facc = 0;
  for (int k = 0; k < b->count; ++k) {
    b->offs[k] = acc;
    b->state_elems[k] = plane_elems(&b->params[k]) * 10;
    acc += b->state_elems[k];
    b->field_offs[k] = facc;
    facc += (long long)b->params[k].nx * b->params[k].ny;
  }
  b->nodes = facc;
  b->state_bytes = round_up((size_t)acc * el, kAlign);
  b->xcd_walk = 2 * b->state_bytes <= kXcdWalkBytes ? 1 : 0;
  // the most items any shape gives: the narrowest strips or the smallest tiles
  b->max_items = std::max(batch_items_for(b, 64, kBatchMinRows, nullptr),
                          batch_items_for(b, 32, 8, nullptr));
  b->off_buf1 = b->state_bytes;
  b->off_doms = 2 * b->state_bytes;
  const size_t dbytes = std::max(hlbm::f32::domain_args_bytes(), hlbm::f64::domain_args_bytes());
  b->off_offs = b->off_doms + round_up(dbytes * b->count, kAlign);
  b->off_foffs = b->off_offs + round_up(sizeof(long long) * b->count, kAlign);
  b->off_items = b->off_foffs + round_up(sizeof(long long) * b->count, kAlign);
  b->off_stat = b->off_items + round_up(sizeof(int) * 4 * (size_t)b->max_items, kAlign);
  b->off_corr = b->off_stat + round_up(sizeof(unsigned) * b->count, kAlign);
  b->total = b->off_corr + round_up(std::max(hlbm::f32::correct_partials_bytes(b->count),
                                             hlbm::f64::correct_partials_bytes(b->count)),
                                    kAlign);
}

int batch_validate(const hlbm_params *p, int32_t count) {
  if (!p || count < 1) return HLBM_EINVAL;
  for (int k = 0; k < count; ++k) {
    if (hlbm_validate(&p[k]) != HLBM_OK) return HLBM_EINVAL;
    if (p[k].dtype != p[0].dtype) return HLBM_EINVAL;
    if (p[k].bc_y == HLBM_BC_WALL) return HLBM_EINVAL;  // the batched step has no wall pass
  }
  return HLBM_OK;
}

bool batch_shape_ok(const hlbm_batch *b, int kind, int tw, int th) {
  if (kind == HLBM_BATCH_TILES)
    return b->dtype == HLBM_F64 ? hlbm::f64::tile_shape_supported(tw, th)
                                : hlbm::f32::tile_shape_supported(tw, th);
  if (kind != HLBM_BATCH_STRIPS) return false;
  if (tw != 64 && tw != 120 && tw != 128 && tw != 184 && tw != 192 && tw != 256) return false;
  if ((tw == 120 || tw == 184) && (b->spl_strips != 2 || b->dtype == HLBM_F64)) return false;
  if (b->spl_strips == 2 && (tw == 256 || (b->dtype == HLBM_F64 && tw == 192)))
    return false;  // the two-step strip kernel's widths
  return th >= kBatchMinRows;
}

// Item list and grids of shape (kind, tw, th); the shape must be one
// batch_shape_ok accepts.
hipError_t batch_upload_items(hlbm_batch *b, int kind, int tw, int th, hipStream_t st) {
  std::vector<int> items;
  items.reserve(4 * (size_t)b->max_items);
  b->nitems = batch_items_for(b, tw, th, &items);
  if (b->nitems > b->max_items) return hipErrorInvalidValue;
  hipError_t e = hipMemcpyAsync(b->ws + b->off_items, items.data(), sizeof(int) * items.size(),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // host vector must outlive the copy
  if (e != hipSuccess) return e;
  b->kind = kind;
  b->tile_w = tw;
  b->tile_h = th;
  const bool tile2 = b->dtype == HLBM_F64 ? hlbm::f64::tile2_shape_supported(tw, th)
                                           : hlbm::f32::tile2_shape_supported(tw, th);
  // the tile kernel takes two steps per launch where the strips would and a
  // two-step tile kernel of this shape exists
  b->spl = kind == HLBM_BATCH_TILES ? (b->spl_strips == 2 && tile2 ? 2 : 1) : b->spl_strips;
  int per_cu1;
  if (kind == HLBM_BATCH_TILES)
    per_cu1 = b->dtype == HLBM_F64 ? hlbm::f64::tile_blocks_per_cu(tw, th)
                                   : hlbm::f32::tile_blocks_per_cu(tw, th);
  else
    per_cu1 = b->dtype == HLBM_F64 ? hlbm::f64::batch_blocks_per_cu(tw)
                                   : hlbm::f32::batch_blocks_per_cu(tw);
  b->grid1 = std::max(1, std::min(b->nitems, per_cu1 * b->ncu));
  b->grid = b->grid1;
  if (b->spl == 2) {
    int per_cu2;
    if (kind == HLBM_BATCH_TILES)
      per_cu2 = b->dtype == HLBM_F64 ? hlbm::f64::tile2_blocks_per_cu(tw, th)
                                     : hlbm::f32::tile2_blocks_per_cu(tw, th);
    else
      per_cu2 = b->dtype == HLBM_F64 ? hlbm::f64::batch2_blocks_per_cu(tw)
                                     : hlbm::f32::batch2_blocks_per_cu(tw);
    b->grid = std::max(1, std::min(b->nitems, per_cu2 * b->ncu));
  }
  for (hipGraphExec_t &g : b->graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  for (hipGraphExec_t &g : b->cgraph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  return hipSuccess;
}

hipError_t batch_launch(hlbm_batch *b, int from, hipStream_t st);

// Ping-pong step pairs per long graph.  Replaying a two-step graph leaves a
// gap of a few microseconds between replays, which for small batches (8 x
// 256^2, then on strips: 23 us per step) cost about 8 %; sixteen steps per
// replay recovered it (21.2 us).
constexpr int kLongPairs = 8;
// Corrected cycles per long closure graph (see hlbm_closure_step).
constexpr int kLongCycles = 8;

// Graph `which` of `pairs` ping-pong pairs from the current buffer (an even
// number of steps leaves the state there), captured on first use and again
// after the current buffer changed; the tile shape's changes destroy it.
hipError_t batch_graph(hlbm_batch *b, int which, int pairs, hipStream_t st) {
  if (b->graph[which] && b->graph_cur[which] == b->cur) return hipSuccess;
  if (b->graph[which]) {
    (void)hipGraphExecDestroy(b->graph[which]);
    b->graph[which] = nullptr;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t el = hipSuccess;
  for (int k = 0; k < pairs && el == hipSuccess; ++k) {
    el = batch_launch(b, b->cur, st);
    if (el == hipSuccess) el = batch_launch(b, b->cur ^ 1, st);
  }
  e = hipStreamEndCapture(st, &g);
  if (el != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return el != hipSuccess ? el : e;
  }
  e = hipGraphInstantiate(&b->graph[which], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph[which] = nullptr;
    return e;
  }
  b->graph_cur[which] = b->cur;
  return hipSuccess;
}

// `mom`: with the tile kernels, the moments of the new state as
// hlbm_batch_moments writes them (rho, u_x, u_y, theta channels of
// b->nodes values each); nullptr for none.
hipError_t batch_launch_spl(hlbm_batch *b, int from, int spl, hipStream_t st,
                            void *mom = nullptr, const hlbm::TileCorr *corr = nullptr) {
  const hlbm::TileCorr none;
  const hlbm::TileCorr &cr = corr ? *corr : none;
  const char *src = b->ws + (from ? b->off_buf1 : 0);
  char *dst = b->ws + (from ? 0 : b->off_buf1);
  const long long *offs = (const long long *)(b->ws + b->off_offs);
  unsigned *stat = (unsigned *)(b->ws + b->off_stat);
  const void *items = b->ws + b->off_items;
  const void *doms = b->ws + b->off_doms;
  const long long *foffs = (const long long *)(b->ws + b->off_foffs);
  if (b->kind == HLBM_BATCH_TILES && spl == 2) {
    if (b->dtype == HLBM_F64)
      return hlbm::f64::step_tile_batch2(doms, offs, items, b->nitems, src, dst, stat,
                                         b->tile_w, b->tile_h, b->grid, b->xcd_walk, mom, foffs,
                                         b->nodes, cr, st);
    return hlbm::f32::step_tile_batch2(doms, offs, items, b->nitems, src, dst, stat, b->tile_w,
                                       b->tile_h, b->grid, b->xcd_walk, mom, foffs, b->nodes, cr,
                                       st);
  }
  if (b->kind == HLBM_BATCH_TILES) {
    if (b->dtype == HLBM_F64)
      return hlbm::f64::step_tile_batch(doms, offs, items, b->nitems, src, dst, stat, b->tile_w,
                                        b->tile_h, b->grid1, b->xcd_walk, mom, foffs, b->nodes,
                                        cr, st);
    return hlbm::f32::step_tile_batch(doms, offs, items, b->nitems, src, dst, stat, b->tile_w,
                                      b->tile_h, b->grid1, b->xcd_walk, mom, foffs, b->nodes, cr,
                                      st);
  }
  if (spl == 2) {
    if (b->dtype == HLBM_F64)
      return hlbm::f64::step_batch2(doms, offs, items, b->nitems, src, dst, stat, b->tile_h,
                                    b->tile_w, b->grid, b->xcd_walk, st);
    return hlbm::f32::step_batch2(doms, offs, items, b->nitems, src, dst, stat, b->tile_h,
                                  b->tile_w, b->grid, b->xcd_walk, st);
  }
  if (b->dtype == HLBM_F64)
    return hlbm::f64::step_batch(doms, offs, items, b->nitems, src, dst, stat, b->tile_h,
                                 b->tile_w, b->grid1, b->xcd_walk, st);
  return hlbm::f32::step_batch(doms, offs, items, b->nitems, src, dst, stat, b->tile_h,
                               b->tile_w, b->grid1, b->xcd_walk, st);
}

// One launch of the batch's kernel (b->spl steps) from buffer `from`.
hipError_t batch_launch(hlbm_batch *b, int from, hipStream_t st) {
  return batch_launch_spl(b, from, b->spl, st);
}

// `n` steps from buffer b->cur, eagerly: launches of b->spl steps, then a
// one-step launch for an odd remainder; advances b->cur (not b->steps).
// Tile kernels only: `mom` goes to the last launch, `corr` to the first
// (see batch_launch_spl).
hipError_t batch_steps_eager(hlbm_batch *b, int n, hipStream_t st, void *mom = nullptr,
                             const hlbm::TileCorr *corr = nullptr) {
  bool first = true;
  for (; n >= b->spl; n -= b->spl) {
    hipError_t e = batch_launch_spl(b, b->cur, b->spl, st, n == b->spl ? mom : nullptr,
                                    first ? corr : nullptr);
    if (e != hipSuccess) return e;
    b->cur ^= 1;
    first = false;
  }
  for (; n > 0; --n) {
    hipError_t e =
        batch_launch_spl(b, b->cur, 1, st, n == 1 ? mom : nullptr, first ? corr : nullptr);
    if (e != hipSuccess) return e;
    b->cur ^= 1;
    first = false;
  }
  return hipSuccess;
}

// Launches batch_steps_eager makes for `n` steps.
int batch_launch_count(const hlbm_batch *b, int n) { return n / b->spl + n % b->spl; }

}  // namespace

extern "C" {

size_t hlbm_batch_workspace_bytes(const hlbm_params *params, int32_t count) {
  if (batch_validate(params, count) != HLBM_OK) return 0;
  hlbm_batch b;
  b.count = count;
  b.dtype = params[0].dtype;
  b.params.assign(params, params + count);
  batch_layout(&b);
  return b.total;
}

int hlbm_batch_init(hlbm_batch **out, const hlbm_params *params, int32_t count, void *workspace,
                    size_t ws_bytes, const void *rho, const void *ux, const void *uy,
                    const void *s, hlbm_stream_t stream) {
  if (!out) return HLBM_EINVAL;
  *out = nullptr;
  if (batch_validate(params, count) != HLBM_OK || !rho || !ux || !uy || !s) return HLBM_EINVAL;
  hlbm_batch *b = new (std::nothrow) hlbm_batch();
  if (!b) return HLBM_ENOMEM;
  b->count = count;
  b->dtype = params[0].dtype;
  b->params.assign(params, params + count);
  batch_layout(b);
  if (!workspace || ws_bytes < b->total || (uintptr_t)workspace % kAlign) {
    delete b;
    return HLBM_EWORKSPACE;
  }
  b->ws = (char *)workspace;
  b->spl_strips = 2;  // two steps per launch when every domain would take them alone
  for (int k = 0; k < count; ++k)
    if (batch_steps_per_launch(&b->params[k]) != 2) b->spl_strips = 1;
  b->spl = b->spl_strips;
  b->doms.resize(count);
  for (int k = 0; k < count; ++k) {
    fill_domain(&b->params[k], &b->doms[k]);
  }
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  // domain table and offsets
  std::vector<char> packed(std::max(hlbm::f32::domain_args_bytes(),
                                    hlbm::f64::domain_args_bytes()) * count);
  if (b->dtype == HLBM_F64)
    hlbm::f64::pack_domains(b->doms.data(), count, packed.data());
  else
    hlbm::f32::pack_domains(b->doms.data(), count, packed.data());
  const size_t dbytes = b->dtype == HLBM_F64 ? hlbm::f64::domain_args_bytes()
                                             : hlbm::f32::domain_args_bytes();
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->ws + b->off_doms, packed.data(), dbytes * count, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->ws + b->off_offs, b->offs.data(), sizeof(long long) * count,
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->ws + b->off_foffs, b->field_offs.data(), sizeof(long long) * count,
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_clear_words, dim3((count + 255) / 256), dim3(256), 0, st,
                       (unsigned *)(b->ws + b->off_stat), count);
    e = hipGetLastError();
  }
  const size_t el = elem_size(b->dtype);
  for (int k = 0; k < count && e == hipSuccess; ++k) {
    const long long fo = b->field_offs[k];
    const char *r = (const char *)rho + fo * el, *u = (const char *)ux + fo * el;
    const char *v = (const char *)uy + fo * el, *sv = (const char *)s + fo * el;
    char *dst = b->ws + b->offs[k] * el;
    e = b->dtype == HLBM_F64 ? hlbm::f64::init(b->doms[k], r, u, v, sv, dst, st)
                             : hlbm::f32::init(b->doms[k], r, u, v, sv, dst, st);
  }
  if (e == hipSuccess) e = batch_upload_items(b, HLBM_BATCH_STRIPS, 128, 32, st);  // synchronises
  if (e != hipSuccess) {
    delete b;
    return HLBM_EHIP;
  }
  *out = b;
  return HLBM_OK;
}

int hlbm_batch_step(hlbm_batch *b, int32_t nsteps, int32_t use_graph, hlbm_stream_t stream) {
  if (!b || nsteps < 0) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (use_graph && !st) return HLBM_EINVAL;  // the legacy null stream cannot be captured
  int n = nsteps;
  if (use_graph) {
    // long graphs while at least kLongPairs pairs of launches remain, then
    // single pairs; the rest runs eagerly
    for (int which = 1; which >= 0; --which) {
      const int len = 2 * (which ? kLongPairs : 1) * b->spl;
      if (n < len) continue;
      if (batch_graph(b, which, len / (2 * b->spl), st) != hipSuccess) return HLBM_EHIP;
      for (; n >= len; n -= len) {
        if (hipGraphLaunch(b->graph[which], st) != hipSuccess) return HLBM_EHIP;
        b->steps += len;
      }
    }
  }
  if (batch_steps_eager(b, n, st) != hipSuccess) return HLBM_EHIP;
  b->steps += n;
  return HLBM_OK;
}

int hlbm_batch_moments(hlbm_batch *b, void *rho, void *ux, void *uy, void *s, void *theta,
                       hlbm_stream_t stream) {
  if (!b) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const char *state = b->ws + (b->cur ? b->off_buf1 : 0);
  long long maxn = 0;
  for (int k = 0; k < b->count; ++k)
    maxn = std::max(maxn, (long long)b->params[k].nx * b->params[k].ny);
  const long long *offs = (const long long *)(b->ws + b->off_offs);
  const long long *foffs = (const long long *)(b->ws + b->off_foffs);
  const void *doms = b->ws + b->off_doms;
  hipError_t e = b->dtype == HLBM_F64
                     ? hlbm::f64::batch_moments(doms, offs, foffs, b->count, maxn, state, rho, ux,
                                                uy, s, theta, st)
                     : hlbm::f32::batch_moments(doms, offs, foffs, b->count, maxn, state, rho, ux,
                                                uy, s, theta, st);
  return hip_status(e);
}

int hlbm_batch_status(hlbm_batch *b, int32_t *host_flags, hlbm_stream_t stream) {
  if (!b) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  std::vector<unsigned> w(b->count);
  if (hipMemcpyAsync(w.data(), b->ws + b->off_stat, sizeof(unsigned) * b->count,
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return HLBM_EHIP;
  int bad = 0;
  for (int k = 0; k < b->count; ++k) {
    if (host_flags) host_flags[k] = w[k] ? 1 : 0;
    bad += w[k] ? 1 : 0;
  }
  return bad;
}

int hlbm_batch_set_shape(hlbm_batch *b, int32_t kernel, int32_t tile_w, int32_t tile_h,
                         hlbm_stream_t stream) {
  if (!b || !batch_shape_ok(b, kernel, tile_w, tile_h)) return HLBM_EINVAL;
  return hip_status(batch_upload_items(b, kernel, tile_w, tile_h, (hipStream_t)stream));
}

int hlbm_batch_set_tile(hlbm_batch *b, int32_t tile_w, int32_t tile_h, hlbm_stream_t stream) {
  return hlbm_batch_set_shape(b, HLBM_BATCH_STRIPS, tile_w, tile_h, stream);
}

int hlbm_batch_autotune(hlbm_batch *b, int32_t steps, void *scratch, int32_t *host_best_kernel,
                        int32_t *host_best_w, int32_t *host_best_h, hlbm_stream_t stream) {
  if (!b || steps < 1 || !scratch) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  // candidate shapes: strips {64, 120, 128, 184, 192, 256} x {4, ..., 128}, then tiles
  struct Shape {
    int kind, w, h;
  };
  std::vector<Shape> cand;
  for (int tw : kBatchTileW)
    for (int th : {4, 8, 16, 32, 64, 128})
      if (batch_shape_ok(b, HLBM_BATCH_STRIPS, tw, th)) cand.push_back({HLBM_BATCH_STRIPS, tw, th});
  for (const auto &t : kTileShapes)
    if (batch_shape_ok(b, HLBM_BATCH_TILES, t[0], t[1]))
      cand.push_back({HLBM_BATCH_TILES, t[0], t[1]});
  if (b->spl_strips == 2 && steps % 2) ++steps;  // whole launches of either kernel
  constexpr int kRepeats = 2;  // best of two timings per shape
  float best = 1e30f;
  Shape bs{b->kind, b->tile_w, b->tile_h};
  const int64_t steps0 = b->steps;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return HLBM_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return HLBM_EHIP;
  }
  // every trial starts from the state at entry, with the divergence flags
  // cleared, so each shape times the same work; the state is restored at the end
  int rc = hlbm_batch_save_state(b, scratch, stream);
  for (const Shape &c : cand) {
    for (int rep = 0; rep < kRepeats && rc == HLBM_OK; ++rep) {
      if (hlbm_batch_load_state(b, scratch, stream) != HLBM_OK) { rc = HLBM_EHIP; break; }
      if (batch_upload_items(b, c.kind, c.w, c.h, st) != hipSuccess) { rc = HLBM_EHIP; break; }
      if (hlbm_batch_step(b, b->spl, 0, st) != HLBM_OK) { rc = HLBM_EHIP; break; }
      if (hipEventRecord(e0, st) != hipSuccess) { rc = HLBM_EHIP; break; }
      if (hlbm_batch_step(b, steps, 0, st) != HLBM_OK) { rc = HLBM_EHIP; break; }
      if (hipEventRecord(e1, st) != hipSuccess) { rc = HLBM_EHIP; break; }
      if (hipEventSynchronize(e1) != hipSuccess) { rc = HLBM_EHIP; break; }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = HLBM_EHIP; break; }
      if (ms < best) {
        best = ms;
        bs = c;
      }
    }
    if (rc != HLBM_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != HLBM_OK) return rc;
  if (hlbm_batch_load_state(b, scratch, stream) != HLBM_OK) return HLBM_EHIP;
  b->steps = steps0;
  if (batch_upload_items(b, bs.kind, bs.w, bs.h, st) != hipSuccess) return HLBM_EHIP;
  if (host_best_kernel) *host_best_kernel = bs.kind;
  if (host_best_w) *host_best_w = bs.w;
  if (host_best_h) *host_best_h = bs.h;
  return HLBM_OK;
}

size_t hlbm_batch_state_bytes(const hlbm_batch *b) { return b ? b->state_bytes : 0; }

int hlbm_batch_save_state(hlbm_batch *b, void *dst, hlbm_stream_t stream) {
  if (!b || !dst) return HLBM_EINVAL;
  return hip_status(hipMemcpyAsync(dst, b->ws + (b->cur ? b->off_buf1 : 0), b->state_bytes,
                                   hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

int hlbm_batch_load_state(hlbm_batch *b, const void *src, hlbm_stream_t stream) {
  if (!b || !src) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(b->ws + (b->cur ? b->off_buf1 : 0), src, b->state_bytes,
                                hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_clear_words, dim3((b->count + 255) / 256), dim3(256), 0, st,
                       (unsigned *)(b->ws + b->off_stat), b->count);
    e = hipGetLastError();
  }
  return hip_status(e);
}

int hlbm_batch_plan(const hlbm_batch *b, int32_t *host_steps_per_launch, int32_t *host_kernel,
                    int32_t *host_tile_w, int32_t *host_tile_h) {
  if (!b || !host_steps_per_launch || !host_kernel || !host_tile_w || !host_tile_h)
    return HLBM_EINVAL;
  *host_steps_per_launch = b->spl;
  *host_kernel = b->kind;
  *host_tile_w = b->tile_w;
  *host_tile_h = b->tile_h;
  return HLBM_OK;
}

int64_t hlbm_batch_nodes(const hlbm_batch *b) { return b ? b->nodes : -1; }

int64_t hlbm_batch_steps_done(const hlbm_batch *b) { return b ? b->steps : -1; }

void hlbm_batch_destroy(hlbm_batch *b) {
  if (!b) return;
  for (hipGraphExec_t g : b->graph)
    if (g) (void)hipGraphExecDestroy(g);
  for (hipGraphExec_t g : b->cgraph)
    if (g) (void)hipGraphExecDestroy(g);
  delete b;
}

}  // extern "C"

// ======================================================================
// Learned-closure coupling
// ======================================================================
namespace {

// every domain of one size, FP32
bool closure_ok(const hlbm_batch *b) {
  if (!b || b->dtype != HLBM_F32) return false;
  for (int k = 1; k < b->count; ++k)
    if (b->params[k].nx != b->params[0].nx || b->params[k].ny != b->params[0].ny) return false;
  return true;
}

hipError_t correct_launch(hlbm_batch *b, const float *x, const float *delta, int conserve,
                          hipStream_t st) {
  char *state = b->ws + (b->cur ? b->off_buf1 : 0);
  const long long n = (long long)b->params[0].nx * b->params[0].ny;
  return hlbm::f32::correct(b->ws + b->off_doms, (const long long *)(b->ws + b->off_offs),
                            b->count, n, state, x, delta, (double *)(b->ws + b->off_corr),
                            conserve, st);
}

// The application half of correct_launch, on sums already taken.
hipError_t correct_apply_launch(hlbm_batch *b, const float *x, const float *delta, int conserve,
                                hipStream_t st) {
  char *state = b->ws + (b->cur ? b->off_buf1 : 0);
  const long long n = (long long)b->params[0].nx * b->params[0].ny;
  return hlbm::f32::correct_apply(b->ws + b->off_doms, (const long long *)(b->ws + b->off_offs),
                                  b->count, n, state, x, delta,
                                  (const double *)(b->ws + b->off_corr), conserve, st);
}

// One corrected cycle: `every` plain steps from buffer b->cur, then the
// network's correction; advances b->cur.  With the strip kernels the
// moments and the correction run as passes of their own.  With the tile
// kernels the cycle's last step writes the moments, and the correction is
// left pending (its sums taken, the state not yet moved): the next cycle's
// first step applies it to the state as it loads it (unless that step is
// also the cycle's last, which overwrites the moments), or closure_flush
// does.  `pending` says on entry whether the previous cycle left one and on
// return whether this one did.  A frozen domain's moments are not refreshed
// and its pending corrections are dropped.
int closure_once(hlbm_batch *b, hlbm_cnn *c, int every, int conserve, hipStream_t st,
                 bool &pending) {
  float *x = hlbm_cnn_io(c, 0), *d = hlbm_cnn_io(c, 1);
  const long long n = (long long)b->params[0].nx * b->params[0].ny;
  const long long N = n * b->count;
  int rc = HLBM_OK;
  if (b->kind == HLBM_BATCH_TILES) {
    hlbm::TileCorr corr;
    if (pending && batch_launch_count(b, every) >= 2) {
      corr.x = x;
      corr.dl = d;
      corr.partials = (const double *)(b->ws + b->off_corr);
      corr.conserve = conserve;
    } else if (pending) {
      if (correct_apply_launch(b, x, d, conserve, st) != hipSuccess) return HLBM_EHIP;
    }
    if (batch_steps_eager(b, every, st, x, corr.x ? &corr : nullptr) != hipSuccess)
      return HLBM_EHIP;
    rc = hlbm_cnn_forward(c, x, n, N, nullptr, b->count, d, n, N, st);
    if (rc != HLBM_OK) return rc;
    if (conserve &&
        hlbm::f32::correct_sums(b->ws + b->off_doms, (const long long *)(b->ws + b->off_offs),
                                b->count, n, x, d, (double *)(b->ws + b->off_corr),
                                st) != hipSuccess)
      return HLBM_EHIP;
    pending = true;
    return HLBM_OK;
  }
  if (batch_steps_eager(b, every, st) != hipSuccess) return HLBM_EHIP;
  rc = hlbm_batch_moments(b, x, x + N, x + 2 * N, nullptr, x + 3 * N, st);
  if (rc != HLBM_OK) return rc;
  rc = hlbm_cnn_forward(c, x, n, N, nullptr, b->count, d, n, N, st);
  if (rc != HLBM_OK) return rc;
  pending = false;
  return correct_launch(b, x, d, conserve, st) == hipSuccess ? HLBM_OK : HLBM_EHIP;
}

// Apply a correction closure_once left pending.
int closure_flush(hlbm_batch *b, hlbm_cnn *c, int conserve, hipStream_t st, bool &pending) {
  if (!pending) return HLBM_OK;
  pending = false;
  return correct_apply_launch(b, hlbm_cnn_io(c, 0), hlbm_cnn_io(c, 1), conserve, st) ==
                 hipSuccess
             ? HLBM_OK
             : HLBM_EHIP;
}

}  // namespace

extern "C" {

int hlbm_batch_correct(hlbm_batch *b, const float *x, const float *delta, int32_t conserve,
                       hlbm_stream_t stream) {
  if (!closure_ok(b) || !x || !delta) return HLBM_EINVAL;
  return hip_status(correct_launch(b, x, delta, conserve ? 1 : 0, (hipStream_t)stream));
}

int hlbm_closure_step(hlbm_batch *b, hlbm_cnn *c, int32_t ncycles, int32_t every,
                      int32_t conserve, int32_t use_graph, hlbm_stream_t stream) {
  if (!closure_ok(b) || !c || ncycles < 0 || every < 1) return HLBM_EINVAL;
  if (hlbm_cnn_max_batch(c) < b->count || hlbm_cnn_ny(c) != b->params[0].ny ||
      hlbm_cnn_nx(c) != b->params[0].nx)
    return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (use_graph && !st) return HLBM_EINVAL;
  conserve = conserve ? 1 : 0;
  int n = ncycles;
  bool pending = false;
  // the graphs start with a pending correction where the cycles leave one:
  // the first cycle then runs eagerly
  const bool fused = b->kind == HLBM_BATCH_TILES;
  if (use_graph && fused && n >= 3) {
    const int rc = closure_once(b, c, every, conserve, st, pending);
    if (rc != HLBM_OK) return rc;
    b->steps += every;
    --n;
  }
  // graphs of kLongCycles cycles while enough remain, then of two (an even
  // count returns the state to the buffer it started from); the rest runs
  // eagerly.  Fewer replays leave fewer gaps between them.
  for (int which = 1; use_graph && which >= 0; --which) {
    const int len = which ? kLongCycles : 2;
    if (n < len) continue;
    hlbm_batch::ClosureKey key;
    key.cur = b->cur;
    key.conserve = conserve;
    key.version = hlbm_cnn_version(c);
    key.every = every;
    key.pending = (int)pending;
    key.net = c;
    hipGraphExec_t &gx = b->cgraph[which];
    if (!gx || !(b->cgraph_key[which] == key)) {
      if (gx) {
        (void)hipGraphExecDestroy(gx);
        gx = nullptr;
      }
      const int cur0 = b->cur;
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return HLBM_EHIP;
      bool gp = pending;
      int rc = HLBM_OK;
      for (int k = 0; k < len && rc == HLBM_OK; ++k)
        rc = closure_once(b, c, every, conserve, st, gp);
      hipError_t e = hipStreamEndCapture(st, &g);
      b->cur = cur0;   // capture only recorded the launches
      if (rc != HLBM_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return HLBM_EHIP;
      }
      e = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        gx = nullptr;
        return HLBM_EHIP;
      }
      b->cgraph_key[which] = key;
    }
    for (; n >= len; n -= len) {
      if (hipGraphLaunch(gx, st) != hipSuccess) return HLBM_EHIP;
      b->steps += (int64_t)len * every;
      pending = fused;  // a replayed cycle leaves a correction pending as an eager one does
    }
  }
  for (; n > 0; --n) {
    const int rc = closure_once(b, c, every, conserve, st, pending);
    if (rc != HLBM_OK) return rc;
    b->steps += every;
  }
  return closure_flush(b, c, conserve, st, pending);
}

}  // extern "C"
