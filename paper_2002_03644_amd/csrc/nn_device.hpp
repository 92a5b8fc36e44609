// Device code of the learned closure: a 3-layer 3x3 convolutional network
// 4 -> 32 -> 32 -> 4 on (rho, u_x, u_y, theta), periodic padding, ReLU after
// the first two layers, trained with a mean-squared-error loss and Adam.
//
// Arithmetic: BF16 operands on the 16x16x32 BF16 matrix cores with FP32
// accumulation; activations and back-propagated gradients stored in BF16;
// master parameters, Adam moments, loss and parameter gradients in FP32.
//
// Layout: activations NHWC [B][H][W][C] in BF16.  Canonical parameters are
// one FP32 vector, per layer the weights [3][3][c_in][c_out] (tap t = 3 dy +
// dx, cross-correlation: out[y][x] = sum in[y + dy - 1][x + dx - 1] w[t])
// followed by the biases [c_out].
//
// Matrix-core operand layout of v_mfma_f32_16x16x32_bf16 (wave of 64):
//   A (16 x 32, M x K): lane m + 16 (k / 8) holds k % 8 of row m;
//   B (32 x 16, K x N): lane n + 16 (k / 8) holds k % 8 of column n;
//   D (16 x 16):        lane n + 16 (m / 4) register m % 4 holds D[m][n].
// Convolutions put output channels on M, pixels on N and (tap, input
// channel) on K, so a B fragment is 8 consecutive channels of one pixel --
// one 16-byte NHWC load -- and a D fragment is 4 consecutive output channels
// of one pixel.
#pragma once

#include <hip/hip_runtime.h>

namespace hlbm {
namespace nn {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 4, kHid = 32, kOut = 4;
// canonical parameter offsets: W1 b1 W2 b2 W3 b3
constexpr int kOffW1 = 0, kOffB1 = 9 * kIn * kHid;              // 1152
constexpr int kOffW2 = kOffB1 + kHid;                            // 1184
constexpr int kOffB2 = kOffW2 + 9 * kHid * kHid;                 // 10400
constexpr int kOffW3 = kOffB2 + kHid;                            // 10432
constexpr int kOffB3 = kOffW3 + 9 * kHid * kOut;                 // 11584
constexpr int kParams = kOffB3 + kOut;                           // 11588

// packed A fragments (bf16x8 per lane), in units of bf16x8
//   scheme "c32": [9 taps][NB][64 lanes], K of one MFMA = 32 input channels
//   scheme "c4":  [2 halves][NB][64 lanes], K = (tap, channel) pairs 0..35
//                 padded to 64, k = 4 t + c
constexpr int kPk1 = 0;                      // layer 1 forward, c4, NB 2
constexpr int kPk2 = kPk1 + 2 * 2 * 64;      // layer 2 forward, c32, NB 2
constexpr int kPk3 = kPk2 + 9 * 2 * 64;      // layer 3 forward, c32, NB 1
constexpr int kPk3T = kPk3 + 9 * 1 * 64;     // layer 3 transposed, c4, NB 2
constexpr int kPk2T = kPk3T + 2 * 2 * 64;    // layer 2 transposed, c32, NB 2
constexpr int kPacked = kPk2T + 9 * 2 * 64;  // total bf16x8 fragments

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ------------------------------------------------------------------ packing
// One packed tensor: either a layer's own weights (forward) or the weights of
// its transposed convolution (backward data: taps flipped, channels swapped,
// W'[t][c][k] = W[8 - t][k][c]).
struct PackDesc {
  int dst;      // first fragment
  int c4;       // 1: scheme c4, 0: scheme c32
  int nb;       // 16-row output blocks
  int cin, cout;            // of the packed convolution
  int src;                  // canonical offset of the layer's weights
  int lcin, lcout;          // the layer's own channel counts
  int transposed;
};

struct PackArgs {
  const float *params;
  bf16 *packed;
  PackDesc d[5];
};

__global__ void k_pack(PackArgs a) {
  const int which = blockIdx.y;
  const PackDesc &p = a.d[which];
  const int nfrag = (p.c4 ? 2 : 9) * p.nb * 64;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nfrag * 8; i += gridDim.x * blockDim.x) {
    const int e = i & 7, frag = i >> 3;
    const int lane = frag & 63, blk = frag >> 6;
    const int nb = blk % p.nb, outer = blk / p.nb;   // outer: tap (c32) or half (c4)
    const int m = lane & 15, g = lane >> 4;
    const int co = 16 * nb + m;
    int t, ci;
    if (p.c4) {
      const int k = 32 * outer + 8 * g + e;
      t = k >> 2;
      ci = k & 3;
    } else {
      t = outer;
      ci = 8 * g + e;
    }
    float v = 0.f;
    if (t < 9 && co < p.cout && ci < p.cin) {
      const int idx = p.transposed ? ((8 - t) * p.lcin + co) * p.lcout + ci
                                   : (t * p.lcin + ci) * p.lcout + co;
      v = a.params[p.src + idx];
    }
    a.packed[(size_t)(p.dst + frag) * 8 + e] = (bf16)v;
  }
}

// ------------------------------------------------------- input standardising
// x raw FP32, element (sample s, channel c, node i) at x[s sb + c sc + i];
// sample s of batch entry b is idx[b] (or b).  Output BF16 NHWC4.
struct PrepArgs {
  const float *x;
  long long sb, sc;
  const int *idx;
  bf16 *out;
  int B, npix;
  float mean[4], inv_std[4];
};

__global__ void k_prep(PrepArgs a) {
  const long long total = (long long)a.B * a.npix;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < total;
       p += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(p / a.npix);
    const long long i = p - (long long)b * a.npix;
    const long long s = a.idx ? a.idx[b] : b;
    const float *src = a.x + s * a.sb + i;
    bf16x4 v;
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (bf16)((src[c * a.sc] - a.mean[c]) * a.inv_std[c]);
    *(bf16x4 *)(a.out + p * 4) = v;
  }
}

// -------------------------------------------------------------- convolution
enum Epilogue { kEpiRelu = 0, kEpiMask = 1, kEpiOut = 2 };

struct ConvArgs {
  const bf16 *in;          // NHWC, CIN channels
  const bf16x8 *wp;        // packed A fragments of this convolution
  const float *bias;       // [COUT] (kEpiRelu, kEpiOut)
  const bf16 *mask;        // NHWC32: ReLU mask source (kEpiMask)
  bf16 *out;               // NHWC32 (kEpiRelu, kEpiMask)
  float *outf;             // kEpiOut: standardised NHWC4, or raw planes
  long long osb, osc;      // kEpiOut raw planes: sample / channel strides; osb 0: NHWC4
  int B, H, W, rows, nsx, nry;
  float os[4], om[4];      // kEpiOut raw: y = clamp(y_std, -clip, clip) * os + om
  float clip;              // kEpiOut raw: bound on |y_std| (0: none)
};

// One wave computes a 16-pixel wide strip of `rows` output rows.  For 32
// input channels each input row is loaded once (three 16-byte loads per lane,
// dx = -1, 0, +1) and feeds the three output rows it touches (taps dy = 0, 1,
// 2), whose accumulators rotate.  For 4 input channels two MFMAs cover the
// 36 (tap, channel) products of one output row.
template <int CIN, int NB, int EPI>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
  const int lane = threadIdx.x & 63;
  const int unit = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (unit >= a.B * a.nsx * a.nry) return;   // wave-uniform
  const int sx = unit % a.nsx;
  const int rest = unit / a.nsx;
  const int ry = rest % a.nry, b = rest / a.nry;
  const int n = lane & 15, g = lane >> 4;
  const int x0 = sx * 16, y0 = ry * a.rows;
  const int R = min(a.rows, a.H - y0);
  const int W = a.W, H = a.H;
  const int xc[3] = {wrap(x0 + n - 1, W), x0 + n, wrap(x0 + n + 1, W)};
  const long long img = (long long)b * H;

  f32x4 init[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = 16 * nb + 4 * g + r;
      init[nb][r] = (EPI != kEpiMask && (EPI != kEpiOut || co < kOut)) ? a.bias[co] : 0.f;
    }
  }

  auto epilogue = [&](const f32x4 *acc, int yo) {
    const long long p = (img + yo) * W + x0 + n;
    if constexpr (EPI == kEpiRelu) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        bf16x4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = (bf16)fmaxf(acc[nb][r], 0.f);
        *(bf16x4 *)(a.out + p * kHid + 16 * nb + 4 * g) = v;
      }
    } else if constexpr (EPI == kEpiMask) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bf16x4 mk = *(const bf16x4 *)(a.mask + p * kHid + 16 * nb + 4 * g);
        bf16x4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = (bf16)((float)mk[r] > 0.f ? acc[nb][r] : 0.f);
        *(bf16x4 *)(a.out + p * kHid + 16 * nb + 4 * g) = v;
      }
    } else {
      if (g == 0) {
        if (a.osb == 0) {
          *(f32x4 *)(a.outf + p * 4) = acc[0];
        } else {
          const long long i = (long long)yo * W + x0 + n;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float ys = a.clip > 0.f ? fminf(fmaxf(acc[0][r], -a.clip), a.clip) : acc[0][r];
            a.outf[b * a.osb + r * a.osc + i] = ys * a.os[r] + a.om[r];
          }
        }
      }
    }
  };

  if constexpr (CIN == kHid) {
    bf16x8 wf[9][NB];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) wf[t][nb] = a.wp[(t * NB + nb) * 64 + lane];
    f32x4 a_prev[NB], a_cur[NB], a_next[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) a_prev[nb] = a_cur[nb] = a_next[nb] = init[nb];
    for (int i = 0; i < R + 2; ++i) {
      const int yin = wrap(y0 - 1 + i, H);
      const bf16 *row = a.in + (img + yin) * W * (long long)kHid + 8 * g;
      bf16x8 bx[3];
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) bx[dx] = *(const bf16x8 *)(row + (long long)xc[dx] * kHid);
      if (i < R) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          a_next[nb] = init[nb];
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) a_next[nb] = mfma(wf[dx][nb], bx[dx], a_next[nb]);
        }
      }
      if (i >= 1 && i <= R) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) a_cur[nb] = mfma(wf[3 + dx][nb], bx[dx], a_cur[nb]);
      }
      if (i >= 2) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int dx = 0; dx < 3; ++dx) a_prev[nb] = mfma(wf[6 + dx][nb], bx[dx], a_prev[nb]);
        epilogue(a_prev, y0 + i - 2);
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        a_prev[nb] = a_cur[nb];
        a_cur[nb] = a_next[nb];
      }
    }
  } else {
    static_assert(CIN == 4, "input channels: 4 or 32");
    bf16x8 wf[2][NB];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) wf[j][nb] = a.wp[(j * NB + nb) * 64 + lane];
    for (int yo = y0; yo < y0 + R; ++yo) {
      f32x4 acc[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[nb] = init[nb];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        bf16x4 h[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int t = 8 * j + 2 * g + e;
          if (t < 9) {
            const int dy = t / 3, dx = t - 3 * dy;
            const int yy = wrap(yo + dy - 1, H);
            h[e] = *(const bf16x4 *)(a.in + ((img + yy) * W + xc[dx]) * 4);
          } else {
            h[e] = bf16x4{(bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f};
          }
        }
        const bf16x8 bv = __builtin_shufflevector(h[0], h[1], 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma(wf[j][nb], bv, acc[nb]);
      }
      epilogue(acc, yo);
    }
  }
}

// ------------------------------------------------------- fused inference
// The three layers in one kernel, activations kept in LDS.  A workgroup owns
// 64 output columns of `rows` rows of one image and works on an 80-column
// region (the 64 columns plus 8 on each side).  Layers 1 and 2 are computed
// on the whole region as five 16-pixel strips; a value at the region's
// outermost column is wrong (its neighbour outside the region is replaced by
// the edge column) and the error moves inwards one column per layer, so
// layer 2 is exact on columns 2..77 and the output layer, computed on the
// four strips covering columns 8..71, is exact.  The standardised input rows
// y0-3 .. y0+rows+2 are staged in LDS first, so the row loop issues no global
// loads.  Layer rows stream through four-row rings: at step j the workgroup
// computes layer-1 row y0+j-3 and completes layer-2 row y0+j-5 and output
// row y0+j-7, with one barrier per step.  Layers 2 and 3 read only the
// newest row of their input ring (three fragments per strip) and add its
// three tap rows to the three output rows it touches, whose accumulators
// rotate; each row still sums its taps in the order t = 0..8.  Each of the
// eight waves has one role, which balances the matrix-core work (18-20
// MFMAs per wave and step: half of what four waves had, so each barrier
// step's serial chain is half as long) and keeps only that role's weights
// in registers:
//   waves 0-4: layer 2, strip = wave      wave 5: layer 1, five strips
//   waves 6-7: output layer, two of its four strips each
// The arithmetic (tap order, FP32 accumulation, BF16 rounding points) is that
// of k_prep and k_conv, so both paths give identical results.
constexpr int kFuseCols = 80, kFuseOut = 64, kFuseWaves = 8, kRing = 4;
constexpr int kFuseMaxRows = 32;
// LDS pixel stride of the layer rings in BF16 elements: 32 channels padded to
// 40 (80 bytes), which spreads the 16-byte reads of a fragment's 16 pixels
// over the LDS banks
constexpr int kPixPad = 40;

struct FusedArgs {
  const float *x;
  long long sb, sc;
  const bf16x8 *wp;        // all packed fragments
  const float *b1, *b2, *b3;
  float *y;
  long long osb, osc;
  int H, W, rows, ncb, nrb;
  float mean[4], inv_std[4], os[4], om[4], clip;
};

// two workgroups per compute unit (LDS allows two): 128 registers per lane
__global__ __launch_bounds__(64 * kFuseWaves) __attribute__((amdgpu_waves_per_eu(4)))
void k_cnn_fused(FusedArgs a) {
  __shared__ __attribute__((aligned(16))) bf16 in_tile[kFuseMaxRows + 6][kFuseCols][4];
  __shared__ __attribute__((aligned(16))) bf16 l1_ring[kRing][kFuseCols][kPixPad];
  __shared__ __attribute__((aligned(16))) bf16 l2_ring[kRing][kFuseCols][kPixPad];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = lane & 15, g = lane >> 4;
  const int cb = blockIdx.x % a.ncb;
  const int rest = blockIdx.x / a.ncb;
  const int rb = rest % a.nrb, b = rest / a.nrb;
  const int H = a.H, W = a.W, R = a.rows;
  const int x0 = cb * kFuseOut, y0 = rb * R;

  // stage the standardised input: tile row q holds image row y0 - 3 + q.
  // Thread t converts the pixels t, t + 512, ... of the (rows + 6) x 80
  // region (a wave covers consecutive columns, so each channel's loads are
  // coalesced); the four channels' loads of all its pixels are issued before
  // the first conversion, so the staging costs one memory latency, and each
  // pixel is one 8-byte LDS write.
  {
    constexpr int kT = 64 * kFuseWaves;
    constexpr int kIt = ((kFuseMaxRows + 6) * kFuseCols + kT - 1) / kT;
    const int npix = (R + 6) * kFuseCols;
    float v[kIt][4];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int p = tid + it * kT;
      if (p < npix) {
        const int q = p / kFuseCols, lc = p - q * kFuseCols;
        int gx = x0 - 8 + lc;
        gx = gx < 0 ? gx + W : (gx >= W ? gx - W : gx);
        int yy = y0 - 3 + q;   // in [-3, H + 2]: one wrap suffices (H >= 4)
        yy = yy < 0 ? yy + H : (yy >= H ? yy - H : yy);
        const float *src = a.x + b * a.sb + (long long)yy * W + gx;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) v[it][ch] = src[ch * a.sc];
      }
    }
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
      const int p = tid + it * kT;
      if (p < npix) {
        const int q = p / kFuseCols, lc = p - q * kFuseCols;
        bf16x4 o;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) o[ch] = (bf16)((v[it][ch] - a.mean[ch]) * a.inv_std[ch]);
        *(bf16x4 *)&in_tile[q][lc][0] = o;
      }
    }
  }
  // a neighbour outside the region reads the edge column instead
  auto clampc = [](int c) { return c < 0 ? 0 : (c >= kFuseCols ? kFuseCols - 1 : c); };
  auto relu_store = [&](bf16 *dst, const f32x4 &acc) {
    bf16x4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = (bf16)fmaxf(acc[r], 0.f);
    *(bf16x4 *)dst = o;
  };

  if (wave < 5) {
    // ---- layer 2 on strip `wave`
    const int col = 16 * wave + n;
    bf16x8 w2[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) w2[t][nb] = a.wp[kPk2 + (t * 2 + nb) * 64 + lane];
    f32x4 bias2[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) bias2[nb][r] = a.b2[16 * nb + 4 * g + r];
    // layer-2 rows in progress: a2m one tap row short, a2o two
    f32x4 a2m[2] = {}, a2o[2] = {};
    for (int j = 1; j <= R + 6; ++j) {
      __syncthreads();
      if (j >= 2 && j <= R + 5) {
        // the newest layer-1 row y0 + j - 4 (written at step j - 1) is read
        // once and gives its tap row dy = 0 to layer-2 row y0 + j - 3
        // (started from the bias), dy = 1 to row y0 + j - 4 and dy = 2 to
        // row y0 + j - 5, which is then complete.  Each row still
        // accumulates its taps in the order t = 0 .. 8.
        const int slot = (j - 1) & 3;
        bf16x8 bv[3];
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
          bv[dx] = *(const bf16x8 *)&l1_ring[slot][clampc(col + dx - 1)][8 * g];
        __builtin_amdgcn_sched_barrier(0);
        f32x4 an[2] = {bias2[0], bias2[1]};
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) {
            an[nb] = mfma(w2[dx][nb], bv[dx], an[nb]);
            a2m[nb] = mfma(w2[3 + dx][nb], bv[dx], a2m[nb]);
            a2o[nb] = mfma(w2[6 + dx][nb], bv[dx], a2o[nb]);
          }
        if (j >= 4) {
#pragma unroll
          for (int nb = 0; nb < 2; ++nb)
            relu_store(&l2_ring[j & 3][col][16 * nb + 4 * g], a2o[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          a2o[nb] = a2m[nb];
          a2m[nb] = an[nb];
        }
      }
    }
  } else if (wave == 5) {
    // ---- layer 1 on the five strips
    bf16x8 w1[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) w1[h][nb] = a.wp[kPk1 + (h * 2 + nb) * 64 + lane];
    f32x4 bias1[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) bias1[nb][r] = a.b1[16 * nb + 4 * g + r];
    for (int j = 1; j <= R + 6; ++j) {
      __syncthreads();
      if (j <= R + 4) {     // layer-1 row y0 + j - 3: tile rows j-1+dy
        for (int st = 0; st < 5; ++st) {
          const int col = 16 * st + n;
          bf16x4 v[2][2];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const int t = 8 * h + 2 * g + e;
              const int tt = t < 9 ? t : 8;
              const int dy = tt / 3, dx = tt - 3 * (tt / 3);
              v[h][e] = *(const bf16x4 *)&in_tile[j - 1 + dy][clampc(col + dx - 1)][0];
              if (t >= 9) v[h][e] = bf16x4{(bf16)0.f, (bf16)0.f, (bf16)0.f, (bf16)0.f};
            }
          __builtin_amdgcn_sched_barrier(0);
          f32x4 acc[2] = {bias1[0], bias1[1]};
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const bf16x8 bv = __builtin_shufflevector(v[h][0], v[h][1], 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) acc[nb] = mfma(w1[h][nb], bv, acc[nb]);
          }
#pragma unroll
          for (int nb = 0; nb < 2; ++nb) relu_store(&l1_ring[j & 3][col][16 * nb + 4 * g], acc[nb]);
        }
      }
    }
  } else {
    // ---- output layer on two of the four strips covering columns 8 .. 71
    const int s0 = 2 * (wave - 6);
    bf16x8 w3[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) w3[t] = a.wp[kPk3 + t * 64 + lane];
    f32x4 bias3;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias3[r] = (4 * g + r < kOut) ? a.b3[4 * g + r] : 0.f;
    // output rows in progress per strip: a3m one tap row short, a3o two
    f32x4 a3m[2] = {}, a3o[2] = {};
    for (int j = 1; j <= R + 6; ++j) {
      __syncthreads();
      if (j < 5) continue;
      // the newest layer-2 row y0 + j - 6 (written at step j - 1) gives tap
      // row dy = 0 to output row y0 + j - 5, dy = 1 to y0 + j - 6 and dy = 2
      // to y0 + j - 7, which is then complete
      const int slot = (j - 1) & 3;
      const long long row = (long long)(y0 + j - 7) * W;
#pragma unroll
      for (int si = 0; si < 2; ++si) {
        const int col = 8 + 16 * (s0 + si) + n;
        bf16x8 bv[3];
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
          bv[dx] = *(const bf16x8 *)&l2_ring[slot][col + dx - 1][8 * g];
        __builtin_amdgcn_sched_barrier(0);
        f32x4 an = bias3;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          an = mfma(w3[dx], bv[dx], an);
          a3m[si] = mfma(w3[3 + dx], bv[dx], a3m[si]);
          a3o[si] = mfma(w3[6 + dx], bv[dx], a3o[si]);
        }
        const f32x4 acc = a3o[si];
        a3o[si] = a3m[si];
        a3m[si] = an;
        if (j >= 7 && g == 0) {
          const long long i = row + x0 + col - 8;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float ys = a.clip > 0.f ? fminf(fmaxf(acc[r], -a.clip), a.clip) : acc[r];
            a.y[b * a.osb + r * a.osc + i] = ys * a.os[r] + a.om[r];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------- weight gradient
// dW[t][ci][co] = sum_p in[p + off(t)][ci] g[p][co], db[co] = sum_p g[p][co]
// over one workgroup's 32-pixel wide, `rw`-row tall patch, written as one
// partial per workgroup.  Pixels run along K, so the patch is staged in LDS
// channel-major: g as [co][row][32], the input as three copies shifted by
// dx = -1, 0, +1, [dx][ci][row][32], which makes every fragment one aligned
// 16-byte LDS read.  Wave w owns the taps of row offset dy = w.
constexpr int kWgTR = 4;   // rows per LDS stage

struct WgradArgs {
  const bf16 *in;     // layer input, NHWC CIN
  const bf16 *grad;   // gradient of the layer output (pre-activation), NHWC COUT
  float *partials;    // [workgroups][9 CIN COUT + COUT]
  int B, H, W, rw, nsx, nry;
};

template <int CIN, int COUT>
__global__ __launch_bounds__(192) void k_wgrad(WgradArgs a) {
  constexpr int TR = kWgTR;
  constexpr int CB = (COUT + 15) / 16, IB = (CIN + 15) / 16;
  constexpr int GV = COUT >= 8 ? 8 : 4, IV = CIN >= 8 ? 8 : 4;   // channels per vector load
  __shared__ __attribute__((aligned(16))) bf16 gt[COUT * TR * 32];
  __shared__ __attribute__((aligned(16))) bf16 at[3 * CIN * (TR + 2) * 32];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int unit = blockIdx.x;
  const int sx = unit % a.nsx;
  const int rest = unit / a.nsx;
  const int ry = rest % a.nry, b = rest / a.nry;
  const int x0 = sx * 32, y0 = ry * a.rw;
  const int W = a.W, H = a.H;
  const long long img = (long long)b * H;
  const int m = lane & 15, g = lane >> 4;

  f32x4 acc[3][CB][IB];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) acc[dx][cb][ib] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbacc[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) dbacc[cb] = 0.f;

  for (int r0 = y0; r0 < y0 + a.rw; r0 += TR) {
    __syncthreads();
    // stage g rows r0 .. r0+TR-1
    for (int it = tid; it < TR * 32 * (COUT / GV); it += 192) {
      const int gi = it % (COUT / GV);
      const int px = it / (COUT / GV);
      const int x = px & 31, rr = px >> 5;
      const bf16 *src = a.grad + ((img + r0 + rr) * W + x0 + x) * COUT + gi * GV;
      if constexpr (GV == 8) {
        const bf16x8 v = *(const bf16x8 *)src;
#pragma unroll
        for (int e = 0; e < 8; ++e) gt[((gi * 8 + e) * TR + rr) * 32 + x] = v[e];
      } else {
        const bf16x4 v = *(const bf16x4 *)src;
#pragma unroll
        for (int e = 0; e < 4; ++e) gt[((gi * 4 + e) * TR + rr) * 32 + x] = v[e];
      }
    }
    // stage input rows r0-1 .. r0+TR, columns x0-1 .. x0+32
    for (int it = tid; it < (TR + 2) * 34 * (CIN / IV); it += 192) {
      const int gi = it % (CIN / IV);
      const int px = it / (CIN / IV);
      const int xp = px % 34, rr = px / 34;
      const int yy = wrap(r0 - 1 + rr, H), xx = wrap(x0 - 1 + xp, W);
      const bf16 *src = a.in + ((img + yy) * W + xx) * CIN + gi * IV;
      bf16 v[IV];
      if constexpr (IV == 8) {
        const bf16x8 t = *(const bf16x8 *)src;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = t[e];
      } else {
        const bf16x4 t = *(const bf16x4 *)src;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = t[e];
      }
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int x = xp - dx;
        if (x >= 0 && x < 32) {
#pragma unroll
          for (int e = 0; e < IV; ++e)
            at[((dx * CIN + gi * IV + e) * (TR + 2) + rr) * 32 + x] = v[e];
        }
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int rr = 0; rr < TR; ++rr) {
      bf16x8 gf[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int co = 16 * cb + m;
        gf[cb] = co < COUT ? *(const bf16x8 *)&gt[(co * TR + rr) * 32 + 8 * g] : bf16x8{};
      }
      if (w == 0) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int e = 0; e < 8; ++e) dbacc[cb] += (float)gf[cb][e];
      }
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
          const int ci = 16 * ib + m;
          const bf16x8 bfr = ci < CIN
              ? *(const bf16x8 *)&at[((dx * CIN + ci) * (TR + 2) + rr + w) * 32 + 8 * g]
              : bf16x8{};
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) acc[dx][cb][ib] = mfma(gf[cb], bfr, acc[dx][cb][ib]);
        }
      }
    }
  }
  constexpr int P = 9 * CIN * COUT + COUT;
  float *out = a.partials + (size_t)unit * P;
  // D[m = co][n = ci]: lane n + 16 q, register r -> co = 16 cb + 4 q + r, ci = 16 ib + n
#pragma unroll
  for (int dx = 0; dx < 3; ++dx)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int ib = 0; ib < IB; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int co = 16 * cb + 4 * g + r, ci = 16 * ib + m;
          if (co < COUT && ci < CIN) out[((w * 3 + dx) * CIN + ci) * COUT + co] = acc[dx][cb][ib][r];
        }
  if (w == 0) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      float s = dbacc[cb];
      s += __shfl_xor(s, 16, 64);
      s += __shfl_xor(s, 32, 64);
      const int co = 16 * cb + m;
      if (g == 0 && co < COUT) out[9 * CIN * COUT + co] = s;
    }
  }
}

// Sum of the per-workgroup partials into the canonical gradient of one
// layer, in two fixed-order passes: workgroup column g sums partials g,
// g + G, g + 2G, ... for 256 parameters, then k_wgrad_final adds the G
// column sums.
constexpr int kWgGroups = 32;

__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *partials, int nparts, int P,
                                                       float *colsum) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  if (j >= P) return;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  int u = g;
  for (; u + 3 * kWgGroups < nparts; u += 4 * kWgGroups) {
    s0 += partials[(size_t)u * P + j];
    s1 += partials[(size_t)(u + kWgGroups) * P + j];
    s2 += partials[(size_t)(u + 2 * kWgGroups) * P + j];
    s3 += partials[(size_t)(u + 3 * kWgGroups) * P + j];
  }
  for (; u < nparts; u += kWgGroups) s0 += partials[(size_t)u * P + j];
  colsum[(size_t)g * P + j] = (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(256) void k_wgrad_final(const float *colsum, int P, float *grad) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= P) return;
  float s = 0.f;
#pragma unroll 8
  for (int g = 0; g < kWgGroups; ++g) s += colsum[(size_t)g * P + j];
  grad[j] = s;
}

// ---------------------------------------------------------------- loss
// d = y_std - (t - om) / os; loss = mean d^2 over all B H W 4 elements;
// g3 = 2 d / N in BF16 NHWC4.  FP64 partial sums per workgroup.
constexpr int kLossThreads = 256;

struct LossArgs {
  const float *y;          // standardised NHWC4
  const float *t;          // raw targets, strided like the inputs
  long long sb, sc;
  const int *idx;
  bf16 *g3;
  double *partials;
  int B, npix;
  float om[4], inv_os[4];
  float scale;             // 2 / N
};

__global__ __launch_bounds__(kLossThreads) void k_loss(LossArgs a) {
  __shared__ double red[kLossThreads / 64];
  const long long total = (long long)a.B * a.npix;
  double acc = 0.0;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < total;
       p += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(p / a.npix);
    const long long i = p - (long long)b * a.npix;
    const long long s = a.idx ? a.idx[b] : b;
    const f32x4 y = *(const f32x4 *)(a.y + p * 4);
    bf16x4 gv;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float tv = (a.t[s * a.sb + c * a.sc + i] - a.om[c]) * a.inv_os[c];
      const float d = y[c] - tv;
      acc += (double)d * d;
      gv[c] = (bf16)(a.scale * d);
    }
    *(bf16x4 *)(a.g3 + p * 4) = gv;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < kLossThreads / 64; ++k) s += red[k];
    a.partials[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(256) void k_loss_final(const double *partials, int nparts,
                                                    double inv_n, float *loss) {
  __shared__ double red[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) s += partials[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *loss = (float)(((red[0] + red[1]) + (red[2] + red[3])) * inv_n);
}

// ---------------------------------------------------------------- Adam
struct AdamArgs {
  float *p, *m, *v;
  const float *g;
  int n;
  float lr, b1, b2, eps, bc1, bc2;   // bc1 = 1 / (1 - b1^t), bc2 = 1 / (1 - b2^t)
};

__global__ void k_adam(AdamArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const float g = a.g[j];
  const float m = a.b1 * a.m[j] + (1.f - a.b1) * g;
  const float v = a.b2 * a.v[j] + (1.f - a.b2) * g * g;
  a.m[j] = m;
  a.v[j] = v;
  a.p[j] -= a.lr * (m * a.bc1) / (sqrtf(v * a.bc2) + a.eps);
}

// ------------------------------------------------------------- restriction
// Block means over f x f cells of mass, momentum and rho theta:
// rho_c = <rho>, u_c = <rho u> / <rho>, theta_c = <rho theta> / <rho>.
struct RestrictArgs {
  const float *rho, *ux, *uy, *th;   // fine planes [B][ny][nx]
  float *out;                        // element (b, c, i) at out[b osb + c osc + i]
  long long osb, osc;
  int B, ny, nx, f;
};

__global__ void k_restrict(RestrictArgs a) {
  const int nyc = a.ny / a.f, nxc = a.nx / a.f;
  const long long total = (long long)a.B * nyc * nxc;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
       q += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(q / ((long long)nyc * nxc));
    const long long ic = q - (long long)b * nyc * nxc;
    const int yc = (int)(ic / nxc), xc = (int)(ic - (long long)yc * nxc);
    float sr = 0.f, su = 0.f, sv = 0.f, st = 0.f;
    for (int dy = 0; dy < a.f; ++dy) {
      const long long row = ((long long)b * a.ny + yc * a.f + dy) * a.nx + xc * a.f;
      for (int dx = 0; dx < a.f; ++dx) {
        const float r = a.rho[row + dx];
        sr += r;
        su += r * a.ux[row + dx];
        sv += r * a.uy[row + dx];
        st += r * a.th[row + dx];
      }
    }
    const float inv = 1.f / sr;
    float *o = a.out + b * a.osb + ic;
    o[0] = sr / (float)(a.f * a.f);
    o[a.osc] = su * inv;
    o[2 * a.osc] = sv * inv;
    o[3 * a.osc] = st * inv;
  }
}

}  // namespace nn
}  // namespace hlbm
