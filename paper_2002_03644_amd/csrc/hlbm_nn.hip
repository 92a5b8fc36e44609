// C ABI of the learned closure (hlbm_nn.h): network handle, workspace
// layout and the launches of the kernels in nn_device.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "hlbm_nn.h"
#include "hlbm_nn_internal.hpp"
#include "nn_device.hpp"

using namespace hlbm::nn;

namespace {

constexpr size_t kAlign = 256;
constexpr int kLossParts = 1024;
constexpr int kConvWaves = 4;   // waves per convolution workgroup

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int wgrad_rows(int B, int H, int W) {
  int rw = 64;
  while (rw > kWgTR && (H % rw != 0 || (long long)B * (W / 32) * (H / rw) < 1024)) rw /= 2;
  return rw;
}

long long wgrad_parts(int B, int H, int W) {
  return (long long)B * (W / 32) * (H / wgrad_rows(B, H, W));
}

constexpr int kPartFloats = 9 * kHid * kHid + kHid;   // largest layer partial

}  // namespace

struct hlbm_cnn {
  int maxb = 0, H = 0, W = 0;
  long long npix = 0;       // H W
  char *ws = nullptr;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  bf16 *packed = nullptr;
  bf16 *xn = nullptr, *a1 = nullptr, *a2 = nullptr, *g3 = nullptr, *g2 = nullptr, *g1 = nullptr;
  float *y = nullptr, *io_x = nullptr, *io_d = nullptr, *wpart = nullptr, *wcol = nullptr;
  double *lpart = nullptr;
  size_t total = 0;
  float norm[16];
  float clip = 0.f;
  int fused = 1;            // inference through k_cnn_fused where the size allows
  int version = 0;          // bumped when launch arguments (norm, clip) change
  long long adam_t = 0;
};

namespace {

void layout(hlbm_cnn *c, char *base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += round_up(bytes, kAlign);
    return p;
  };
  const size_t px = (size_t)c->maxb * c->npix;
  long long parts = 0;
  for (int b = 1; b <= c->maxb; ++b) parts = std::max(parts, wgrad_parts(b, c->H, c->W));
  c->params = (float *)take(sizeof(float) * kParams);
  c->grads = (float *)take(sizeof(float) * kParams);
  c->m = (float *)take(sizeof(float) * kParams);
  c->v = (float *)take(sizeof(float) * kParams);
  c->packed = (bf16 *)take(sizeof(bf16) * 8 * kPacked);
  c->xn = (bf16 *)take(sizeof(bf16) * 4 * px);
  c->a1 = (bf16 *)take(sizeof(bf16) * kHid * px);
  c->a2 = (bf16 *)take(sizeof(bf16) * kHid * px);
  c->y = (float *)take(sizeof(float) * 4 * px);
  c->g3 = (bf16 *)take(sizeof(bf16) * 4 * px);
  c->g2 = (bf16 *)take(sizeof(bf16) * kHid * px);
  c->g1 = (bf16 *)take(sizeof(bf16) * kHid * px);
  c->wpart = (float *)take(sizeof(float) * kPartFloats * (size_t)parts);
  c->wcol = (float *)take(sizeof(float) * kPartFloats * (size_t)kWgGroups);
  c->lpart = (double *)take(sizeof(double) * kLossParts + sizeof(float));
  c->io_x = (float *)take(sizeof(float) * 4 * px);
  c->io_d = (float *)take(sizeof(float) * 4 * px);
  c->total = off;
}

bool valid_dims(int32_t maxb, int32_t ny, int32_t nx) {
  if (maxb < 1 || ny < 4 || nx < 32 || nx % 32 || ny % 4) return false;
  return (long long)maxb * nx * ny < (1LL << 31);
}

int hip_status(hipError_t e) { return e == hipSuccess ? HLBM_OK : HLBM_EHIP; }

int grid_for(long long n, int threads) {
  long long b = (n + threads - 1) / threads;
  return (int)std::max(1LL, std::min(b, 65536LL));
}

hipError_t pack(hlbm_cnn *c, hipStream_t st) {
  PackArgs a;
  a.params = c->params;
  a.packed = c->packed;
  //                dst    c4 nb cin   cout  src     lcin  lcout transposed
  a.d[0] = PackDesc{kPk1, 1, 2, kIn, kHid, kOffW1, kIn, kHid, 0};
  a.d[1] = PackDesc{kPk2, 0, 2, kHid, kHid, kOffW2, kHid, kHid, 0};
  a.d[2] = PackDesc{kPk3, 0, 1, kHid, kOut, kOffW3, kHid, kOut, 0};
  a.d[3] = PackDesc{kPk3T, 1, 2, kOut, kHid, kOffW3, kHid, kOut, 1};
  a.d[4] = PackDesc{kPk2T, 0, 2, kHid, kHid, kOffW2, kHid, kHid, 1};
  hipLaunchKernelGGL(k_pack, dim3(32, 5), dim3(256), 0, st, a);
  return hipGetLastError();
}

// rows per wave: a divisor of H (a multiple of 4), halved until the launch
// has enough waves to fill the chip
int conv_rows(int B, int H, int W) {
  int rows = 16;
  while (rows > 4 && (H % rows != 0 || (long long)B * (W / 16) * (H / rows) < 4096)) rows /= 2;
  return rows;
}

template <int CIN, int NB, int EPI>
hipError_t conv(hlbm_cnn *c, int B, const bf16 *in, int pk, const float *bias, const bf16 *mask,
                bf16 *out, float *outf, long long osb, long long osc, hipStream_t st) {
  ConvArgs a;
  a.in = in;
  a.wp = (const bf16x8 *)c->packed + pk;
  a.bias = bias;
  a.mask = mask;
  a.out = out;
  a.outf = outf;
  a.osb = osb;
  a.osc = osc;
  a.B = B;
  a.H = c->H;
  a.W = c->W;
  a.rows = conv_rows(B, c->H, c->W);
  a.nsx = c->W / 16;
  a.nry = (c->H + a.rows - 1) / a.rows;
  for (int k = 0; k < 4; ++k) {
    a.om[k] = c->norm[8 + k];
    a.os[k] = c->norm[12 + k];
  }
  a.clip = c->clip;
  const long long units = (long long)B * a.nsx * a.nry;
  hipLaunchKernelGGL((k_conv<CIN, NB, EPI>), dim3((units + kConvWaves - 1) / kConvWaves),
                     dim3(64 * kConvWaves), 0, st, a);
  return hipGetLastError();
}

template <int CIN, int COUT>
hipError_t wgrad(hlbm_cnn *c, int B, const bf16 *in, const bf16 *g, int off, hipStream_t st) {
  WgradArgs a;
  a.in = in;
  a.grad = g;
  a.partials = c->wpart;
  a.B = B;
  a.H = c->H;
  a.W = c->W;
  a.rw = wgrad_rows(B, c->H, c->W);
  a.nsx = c->W / 32;
  a.nry = c->H / a.rw;
  const int parts = B * a.nsx * a.nry;
  hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(parts), dim3(192), 0, st, a);
  constexpr int P = 9 * CIN * COUT + COUT;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((P + 255) / 256, kWgGroups), dim3(256), 0, st,
                     (const float *)c->wpart, parts, P, c->wcol);
  hipLaunchKernelGGL(k_wgrad_final, dim3((P + 255) / 256), dim3(256), 0, st,
                     (const float *)c->wcol, P, c->grads + off);
  return hipGetLastError();
}

hipError_t prep(hlbm_cnn *c, const float *x, long long sb, long long sc, const int32_t *idx,
                int B, hipStream_t st) {
  PrepArgs a;
  a.x = x;
  a.sb = sb;
  a.sc = sc;
  a.idx = idx;
  a.out = c->xn;
  a.B = B;
  a.npix = (int)c->npix;
  for (int k = 0; k < 4; ++k) {
    a.mean[k] = c->norm[k];
    a.inv_std[k] = 1.f / c->norm[4 + k];
  }
  hipLaunchKernelGGL(k_prep, dim3(grid_for((long long)B * c->npix, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

// layers 1 and 2; layer 3 is launched by the caller with its own epilogue
hipError_t hidden(hlbm_cnn *c, int B, hipStream_t st) {
  hipError_t e = conv<kIn, 2, kEpiRelu>(c, B, c->xn, kPk1, c->params + kOffB1, nullptr, c->a1,
                                        nullptr, 0, 0, st);
  if (e == hipSuccess)
    e = conv<kHid, 2, kEpiRelu>(c, B, c->a1, kPk2, c->params + kOffB2, nullptr, c->a2, nullptr,
                                0, 0, st);
  return e;
}

// rows per workgroup of the fused kernel: a divisor of H (a multiple of 4),
// halved until there are two workgroups per compute unit; 0 if the width
// does not tile by 64 columns
int fused_rows(int B, int H, int W) {
  if (W % kFuseOut) return 0;
  int R = kFuseMaxRows;
  while (R > 4 && (H % R != 0 || (long long)B * (W / kFuseOut) * (H / R) < 512)) R /= 2;
  return H % R == 0 ? R : 0;
}

hipError_t fused_forward(hlbm_cnn *c, const float *x, long long sb, long long sc, int B, float *y,
                         long long osb, long long osc, int R, hipStream_t st) {
  FusedArgs a;
  a.x = x;
  a.sb = sb;
  a.sc = sc;
  a.wp = (const bf16x8 *)c->packed;
  a.b1 = c->params + kOffB1;
  a.b2 = c->params + kOffB2;
  a.b3 = c->params + kOffB3;
  a.y = y;
  a.osb = osb;
  a.osc = osc;
  a.H = c->H;
  a.W = c->W;
  a.rows = R;
  a.ncb = c->W / kFuseOut;
  a.nrb = c->H / R;
  for (int k = 0; k < 4; ++k) {
    a.mean[k] = c->norm[k];
    a.inv_std[k] = 1.f / c->norm[4 + k];
    a.om[k] = c->norm[8 + k];
    a.os[k] = c->norm[12 + k];
  }
  a.clip = c->clip;
  hipLaunchKernelGGL(k_cnn_fused, dim3(B * a.ncb * a.nrb), dim3(64 * kFuseWaves), 0, st, a);
  return hipGetLastError();
}

bool args_ok(const hlbm_cnn *c, const float *x, int32_t B) {
  return c && x && B >= 1 && B <= c->maxb;
}

}  // namespace

// ---------------------------------------------------------------- internal
float *hlbm_cnn_io(hlbm_cnn *c, int which) { return which ? c->io_d : c->io_x; }
int hlbm_cnn_max_batch(const hlbm_cnn *c) { return c->maxb; }
int hlbm_cnn_ny(const hlbm_cnn *c) { return c->H; }
int hlbm_cnn_nx(const hlbm_cnn *c) { return c->W; }
int hlbm_cnn_version(const hlbm_cnn *c) { return c->version; }

extern "C" {

size_t hlbm_cnn_workspace_bytes(int32_t max_batch, int32_t ny, int32_t nx) {
  if (!valid_dims(max_batch, ny, nx)) return 0;
  hlbm_cnn c;
  c.maxb = max_batch;
  c.H = ny;
  c.W = nx;
  c.npix = (long long)ny * nx;
  layout(&c, nullptr);
  return c.total;
}

int hlbm_cnn_init(hlbm_cnn **out, int32_t max_batch, int32_t ny, int32_t nx, void *workspace,
                  size_t ws_bytes, const float *params, hlbm_stream_t stream) {
  if (!out) return HLBM_EINVAL;
  *out = nullptr;
  if (!valid_dims(max_batch, ny, nx) || !params) return HLBM_EINVAL;
  hlbm_cnn *c = new (std::nothrow) hlbm_cnn();
  if (!c) return HLBM_ENOMEM;
  c->maxb = max_batch;
  c->H = ny;
  c->W = nx;
  c->npix = (long long)ny * nx;
  layout(c, nullptr);
  if (!workspace || ws_bytes < c->total || (uintptr_t)workspace % kAlign) {
    delete c;
    return HLBM_EWORKSPACE;
  }
  c->ws = (char *)workspace;
  layout(c, c->ws);
  for (int k = 0; k < 4; ++k) {
    c->norm[k] = 0.f;
    c->norm[4 + k] = 1.f;
    c->norm[8 + k] = 0.f;
    c->norm[12 + k] = 1.f;
  }
  const int rc = hlbm_cnn_set_params(c, params, stream);
  if (rc != HLBM_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return HLBM_OK;
}

int hlbm_cnn_set_params(hlbm_cnn *c, const float *params, hlbm_stream_t stream) {
  if (!c || !params) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(c->params, params, sizeof(float) * kParams,
                                hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(c->m, 0, sizeof(float) * kParams, st);
  if (e == hipSuccess) e = hipMemsetAsync(c->v, 0, sizeof(float) * kParams, st);
  if (e == hipSuccess) e = hipMemsetAsync(c->grads, 0, sizeof(float) * kParams, st);
  if (e == hipSuccess) e = pack(c, st);
  c->adam_t = 0;
  return hip_status(e);
}

int hlbm_cnn_get_params(hlbm_cnn *c, float *dst, hlbm_stream_t stream) {
  if (!c || !dst) return HLBM_EINVAL;
  return hip_status(hipMemcpyAsync(dst, c->params, sizeof(float) * kParams,
                                   hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

int hlbm_cnn_get_grads(hlbm_cnn *c, float *dst, hlbm_stream_t stream) {
  if (!c || !dst) return HLBM_EINVAL;
  return hip_status(hipMemcpyAsync(dst, c->grads, sizeof(float) * kParams,
                                   hipMemcpyDeviceToDevice, (hipStream_t)stream));
}

int hlbm_cnn_set_norm(hlbm_cnn *c, const float *host_norm) {
  if (!c || !host_norm) return HLBM_EINVAL;
  for (int k = 0; k < 16; ++k)
    if (!std::isfinite(host_norm[k])) return HLBM_EINVAL;
  for (int k = 0; k < 4; ++k)
    if (!(host_norm[4 + k] > 0.f) || !(host_norm[12 + k] > 0.f)) return HLBM_EINVAL;
  std::copy(host_norm, host_norm + 16, c->norm);
  ++c->version;
  return HLBM_OK;
}

int hlbm_cnn_set_output_clip(hlbm_cnn *c, float clip) {
  if (!c || !(clip >= 0.f) || !std::isfinite(clip)) return HLBM_EINVAL;
  c->clip = clip;
  ++c->version;
  return HLBM_OK;
}

int hlbm_cnn_set_fused(hlbm_cnn *c, int32_t enable) {
  if (!c) return HLBM_EINVAL;
  c->fused = enable ? 1 : 0;
  ++c->version;
  return HLBM_OK;
}

int hlbm_cnn_forward(hlbm_cnn *c, const float *x, int64_t x_sstride, int64_t x_cstride,
                     const int32_t *idx, int32_t batch, float *y, int64_t y_sstride,
                     int64_t y_cstride, hlbm_stream_t stream) {
  if (!args_ok(c, x, batch) || !y || y_sstride <= 0 || y_cstride <= 0) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int R = fused_rows(batch, c->H, c->W);
  if (c->fused && R > 0 && !idx)
    return hip_status(fused_forward(c, x, x_sstride, x_cstride, batch, y, y_sstride, y_cstride,
                                    R, st));
  hipError_t e = prep(c, x, x_sstride, x_cstride, idx, batch, st);
  if (e == hipSuccess) e = hidden(c, batch, st);
  if (e == hipSuccess)
    e = conv<kHid, 1, kEpiOut>(c, batch, c->a2, kPk3, c->params + kOffB3, nullptr, nullptr, y,
                               y_sstride, y_cstride, st);
  return hip_status(e);
}

int hlbm_cnn_loss_grad(hlbm_cnn *c, const float *x, int64_t x_sstride, int64_t x_cstride,
                       const float *target, int64_t t_sstride, int64_t t_cstride,
                       const int32_t *idx, int32_t batch, float *loss, hlbm_stream_t stream) {
  if (!args_ok(c, x, batch) || !target) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int B = batch;
  hipError_t e = prep(c, x, x_sstride, x_cstride, idx, B, st);
  if (e == hipSuccess) e = hidden(c, B, st);
  if (e == hipSuccess)   // standardised output, NHWC4
    e = conv<kHid, 1, kEpiOut>(c, B, c->a2, kPk3, c->params + kOffB3, nullptr, nullptr, c->y, 0,
                               0, st);
  if (e != hipSuccess) return HLBM_EHIP;
  LossArgs la;
  la.y = c->y;
  la.t = target;
  la.sb = t_sstride;
  la.sc = t_cstride;
  la.idx = idx;
  la.g3 = c->g3;
  la.partials = c->lpart;
  la.B = B;
  la.npix = (int)c->npix;
  const double nel = 4.0 * B * (double)c->npix;
  for (int k = 0; k < 4; ++k) {
    la.om[k] = c->norm[8 + k];
    la.inv_os[k] = 1.f / c->norm[12 + k];
  }
  la.scale = (float)(2.0 / nel);
  const int parts = std::min(kLossParts, grid_for((long long)B * c->npix, kLossThreads));
  hipLaunchKernelGGL(k_loss, dim3(parts), dim3(kLossThreads), 0, st, la);
  if (loss)
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, (const double *)c->lpart, parts,
                       1.0 / nel, loss);
  e = hipGetLastError();
  // layer 3: weights from (a2, g3); back to layer 2 through the ReLU of a2
  if (e == hipSuccess) e = wgrad<kHid, kOut>(c, B, c->a2, c->g3, kOffW3, st);
  if (e == hipSuccess)
    e = conv<kOut, 2, kEpiMask>(c, B, c->g3, kPk3T, nullptr, c->a2, c->g2, nullptr, 0, 0, st);
  // layer 2: weights from (a1, g2); back to layer 1 through the ReLU of a1
  if (e == hipSuccess) e = wgrad<kHid, kHid>(c, B, c->a1, c->g2, kOffW2, st);
  if (e == hipSuccess)
    e = conv<kHid, 2, kEpiMask>(c, B, c->g2, kPk2T, nullptr, c->a1, c->g1, nullptr, 0, 0, st);
  // layer 1: weights from (xn, g1)
  if (e == hipSuccess) e = wgrad<kIn, kHid>(c, B, c->xn, c->g1, kOffW1, st);
  return hip_status(e);
}

int hlbm_cnn_adam(hlbm_cnn *c, float lr, hlbm_stream_t stream) {
  if (!c || !(lr >= 0.f)) return HLBM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const long long t = c->adam_t + 1;
  AdamArgs a;
  a.p = c->params;
  a.m = c->m;
  a.v = c->v;
  a.g = c->grads;
  a.n = kParams;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.bc1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)t)));
  a.bc2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)t)));
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = pack(c, st);
  if (e != hipSuccess) return HLBM_EHIP;
  c->adam_t = t;
  return (int)std::min<long long>(t, 0x7fffffff);
}

int hlbm_cnn_train_step(hlbm_cnn *c, const float *x, int64_t x_sstride, int64_t x_cstride,
                        const float *target, int64_t t_sstride, int64_t t_cstride,
                        const int32_t *idx, int32_t batch, float lr, float *loss,
                        hlbm_stream_t stream) {
  const int rc = hlbm_cnn_loss_grad(c, x, x_sstride, x_cstride, target, t_sstride, t_cstride,
                                    idx, batch, loss, stream);
  if (rc != HLBM_OK) return rc;
  const int t = hlbm_cnn_adam(c, lr, stream);
  return t < 0 ? t : HLBM_OK;
}

void hlbm_cnn_destroy(hlbm_cnn *c) { delete c; }

int hlbm_restrict(const float *rho, const float *ux, const float *uy, const float *theta,
                  int32_t batch, int32_t ny, int32_t nx, int32_t factor, float *out,
                  int64_t o_sstride, int64_t o_cstride, hlbm_stream_t stream) {
  if (!rho || !ux || !uy || !theta || !out || batch < 1 || factor < 1 || ny < factor ||
      nx < factor || ny % factor || nx % factor || o_sstride <= 0 || o_cstride <= 0)
    return HLBM_EINVAL;
  RestrictArgs a;
  a.rho = rho;
  a.ux = ux;
  a.uy = uy;
  a.th = theta;
  a.out = out;
  a.osb = o_sstride;
  a.osc = o_cstride;
  a.B = batch;
  a.ny = ny;
  a.nx = nx;
  a.f = factor;
  const long long n = (long long)batch * (ny / factor) * (nx / factor);
  hipLaunchKernelGGL(k_restrict, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, a);
  return hip_status(hipGetLastError());
}

}  // extern "C"
