// C ABI of the hybrid LBM library (declared in include/hlbm.h): parameter
// validation, workspace layout, launches and status codes.  The workspace is
// the caller's device buffer; this file never allocates device memory.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "hlbm.h"
#include "hlbm_launch.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr double kCs2 = 1.0 / 3.0;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_size(int dtype) { return dtype == HLBM_F64 ? 8 : 4; }

long long plane_elems(const hlbm_params *p) {
  return (long long)round_up((size_t)p->nx * (size_t)p->ny, 64);
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
  hlbm::TileShape tile;
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
// storage, from the nine Hermite coefficients of the rest equilibrium.
void rest_equilibrium(double rho, double theta, double f[9]) {
  const double c = kCs2 * (theta - 1.0);
  const double A0 = rho, Axx = rho * c, Ayy = rho * c, Axxyy = rho * c * c;
  f[0] = 4.0 / 9.0 * (A0 - 1.5 * (Axx + Ayy) + 2.25 * Axxyy);
  const double bx = A0 + 3 * Axx - 1.5 * Ayy - 4.5 * Axxyy;
  f[1] = f[3] = bx / 9.0;
  const double by = A0 + 3 * Ayy - 1.5 * Axx - 4.5 * Axxyy;
  f[2] = f[4] = by / 9.0;
  const double bd = A0 + 3 * (Axx + Ayy) + 9 * Axxyy;
  f[5] = f[6] = f[7] = f[8] = bd / 36.0;
}

hlbm::TileShape default_tile(const hlbm_params *p) {
  hlbm::TileShape t;
  // 128-column tiles with 32-row strips measured fastest at 8192^2 in FP32
  // (aligned row segments, 21 resident waves per CU).
  t.bw = p->tile_w ? p->tile_w : 128;
  int rows = p->tile_h ? p->tile_h : 32;
  if (rows > p->ny) rows = p->ny;
  t.rows = rows;
  t.xcd_remap = 1;
  return t;
}

void fill_domain(const hlbm_params *p, hlbm::HostDomain *d) {
  memset(d, 0, sizeof(*d));
  d->plane = plane_elems(p);
  d->nx = p->nx;
  d->ny = p->ny;
  d->bcx = p->bc_x;
  d->bcy = p->bc_y;
  d->flags = (p->phi_mode == HLBM_PHI_FD ? 1 : 0) | (p->e1_centred ? 2 : 0) | (p->e2_off ? 4 : 0);
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
  if (p->dtype == HLBM_F32) {
    d->rho_ref = p->rho_ref;
    d->theta_ref = p->theta_ref;
    d->log_rho_ref = log(p->rho_ref);
    d->s_ref = cv * log(p->theta_ref / pow(p->rho_ref, g - 1.0));
    rest_equilibrium(p->rho_ref, p->theta_ref, d->fref);
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
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 1) return HLBM_EINVAL;
  if (p->dtype != HLBM_F64 && p->dtype != HLBM_F32) return HLBM_EINVAL;
  if (p->phi_mode != HLBM_PHI_LBM && p->phi_mode != HLBM_PHI_FD) return HLBM_EINVAL;
  if (p->e1_centred < 0 || p->e1_centred > 1 || p->e2_off < 0 || p->e2_off > 1) return HLBM_EINVAL;
  if (p->tile_w != 0 && p->tile_w != 64 && p->tile_w != 128 && p->tile_w != 256) return HLBM_EINVAL;
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
  fill_domain(p, &h->dom);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (p->dtype == HLBM_F64)
    e = hlbm::f64::init(h->dom, rho, ux, uy, s, buf(h, 0), st);
  else
    e = hlbm::f32::init(h->dom, rho, ux, uy, s, buf(h, 0), st);
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
  for (int32_t n = 0; n < nsteps; ++n) {
    hipError_t e;
    if (h->p.dtype == HLBM_F64)
      e = hlbm::f64::step(h->dom, buf(h, h->cur), buf(h, h->cur ^ 1), status_word(h), h->tile, st);
    else
      e = hlbm::f32::step(h->dom, buf(h, h->cur), buf(h, h->cur ^ 1), status_word(h), h->tile, st);
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
