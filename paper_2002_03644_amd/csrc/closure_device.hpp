// Coupling of the learned correction to a batch of HLBM domains (one
// precision; included after hlbm_device.hpp).
//
// Given the moments X = (rho, u_x, u_y, theta) of every node and a predicted
// increment D = (d_rho, d_ux, d_uy, d_theta), the corrected state is
//   rho'   = rho + d_rho - a,                       a = <d_rho>
//   rho'u' = rho' (u + d_u) - b,  b = <(rho + d_rho)(u + d_u) - rho u> - a <u + d_u>
//   theta' = theta + d_theta
// (with a = b = 0 when conservation is not asked for), so that the domain's
// total mass and momentum are unchanged.  Only the equilibrium part of the
// populations moves: F_i <- F_i + f^eq_i(X') - f^eq_i(X), which keeps the
// non-equilibrium part F - f^eq, and the entropy follows the new state,
// s' = s + c_v [ln(theta'/theta) - (gamma - 1) ln(rho'/rho)].
#pragma once

namespace hlbm {
namespace HLBM_NS {

constexpr int kCorrThreads = 256;
constexpr int kCorrParts = 64;   // partial-sum workgroups per domain
constexpr int kCorrVals = 5;     // sum d_rho, sum dm_x, sum dm_y, sum u'_x, sum u'_y

struct CorrArgs {
  const DomainArgs *doms;
  const long long *offs;   // element offset of each domain's state in the buffer
  real *state;             // buffer holding the current state
  const float *x, *dl;     // element (channel c, domain k, node i) at [c sc + k n + i]
  long long n, sc;
  double *partials;        // [domains][kCorrParts][kCorrVals]
  int conserve;
};

__global__ __launch_bounds__(kCorrThreads) void k_corr_sums(CorrArgs a) {
  __shared__ double red[kCorrThreads / 64][kCorrVals];
  const int k = blockIdx.y;
  const long long base = (long long)k * a.n;
  double s[kCorrVals] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long i = blockIdx.x * (long long)kCorrThreads + threadIdx.x; i < a.n;
       i += (long long)kCorrParts * kCorrThreads) {
    const double r = a.x[base + i], u = a.x[a.sc + base + i], v = a.x[2 * a.sc + base + i];
    const double dr = a.dl[base + i], du = a.dl[a.sc + base + i], dv = a.dl[2 * a.sc + base + i];
    s[0] += dr;
    s[1] += (r + dr) * (u + du) - r * u;
    s[2] += (r + dr) * (v + dv) - r * v;
    s[3] += u + du;
    s[4] += v + dv;
  }
#pragma unroll
  for (int q = 0; q < kCorrVals; ++q) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off, 64);
  }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < kCorrVals; ++q) red[threadIdx.x >> 6][q] = s[q];
  __syncthreads();
  if (threadIdx.x < kCorrVals) {
    double t = 0.0;
    for (int w = 0; w < kCorrThreads / 64; ++w) t += red[w][threadIdx.x];
    a.partials[((long long)k * kCorrParts + blockIdx.x) * kCorrVals + threadIdx.x] = t;
  }
}

// Total q of domain k over its kCorrParts partial sums, in a fixed order.
__device__ __forceinline__ double corr_total(const double *partials, int k, int q) {
  double t = 0.0;
  for (int j = 0; j < kCorrParts; ++j) t += partials[((long long)k * kCorrParts + j) * kCorrVals + q];
  return t;
}

// The domain's conservation shifts a (density) and b (momentum) from its
// totals (zero when conservation is not asked for), for n nodes.
struct CorrShift {
  real sa, bx, by;
};
__device__ __forceinline__ CorrShift corr_shift(const double *tot, long long n, int conserve) {
  const double inv_n = 1.0 / (double)n;
  const double am = conserve ? tot[0] * inv_n : 0.0;
  CorrShift c;
  c.sa = (real)am;
  c.bx = conserve ? (real)((tot[1] - am * tot[3]) * inv_n) : real(0);
  c.by = conserve ? (real)((tot[2] - am * tot[4]) * inv_n) : real(0);
  return c;
}

// Hermite coefficients of f^eq(rho, u, theta) that the projection needs,
// c = c_s^2 (theta - 1).
struct EqCoef {
  real A0, Ax, Ay, Axx, Axy, Ayy, Axxy, Axyy, Axxyy;
};

__device__ __forceinline__ EqCoef eq_coef(real r, real u, real v, real th) {
  const real c = real(kCs2) * (th - real(1));
  const real rc = r * c;
  EqCoef e;
  e.A0 = r;
  e.Ax = r * u;
  e.Ay = r * v;
  e.Axx = r * u * u + rc;
  e.Ayy = r * v * v + rc;
  e.Axy = r * u * v;
  e.Axxy = r * u * u * v + rc * v;
  e.Axyy = r * u * v * v + rc * u;
  e.Axxyy = r * u * u * v * v + rc * (u * u + v * v) + rc * c;
  return e;
}

// The correction of one node: x, dl point at the node's domain in the
// moments and increments (channel stride sc), i is its dense index.  Its
// populations move by df, its entropy sv to corr_s(sv, q).  Shared by
// k_corr_apply and the tile kernels, which apply a pending correction to
// the state they load (identical arithmetic, so identical results).
struct CorrDelta {
  real df[kQ];
  real cv, ls;  // the entropy moves by cv ls
};

__device__ __forceinline__ CorrDelta corr_delta(const DomainArgs &d, const float *x,
                                                const float *dl, long long sc, long long i,
                                                const CorrShift &c) {
  const real r = x[i], u = x[sc + i];
  const real v = x[2 * sc + i], th = x[3 * sc + i];
  const real dr = dl[i], du = dl[sc + i];
  const real dv = dl[2 * sc + i], dth = dl[3 * sc + i];
  const real r2 = r + dr - c.sa;
  const real inv_r2 = real(1) / r2;
  const real u2 = (u + du) - c.bx * inv_r2, v2 = (v + dv) - c.by * inv_r2;
  const real th2 = th + dth;
  const EqCoef e1 = eq_coef(r, u, v, th), e2 = eq_coef(r2, u2, v2, th2);
  CorrDelta q;
  const real dxxyy = (d.flags & kFlagFeq3) ? real(0) : e2.Axxyy - e1.Axxyy;
  project(e2.A0 - e1.A0, e2.Ax - e1.Ax, e2.Ay - e1.Ay, e2.Axx - e1.Axx, e2.Axy - e1.Axy,
          e2.Ayy - e1.Ayy, e2.Axxy - e1.Axxy, e2.Axyy - e1.Axyy, dxxyy, q.df);
  q.cv = real(1) / d.inv_cv;
  q.ls = log_r(th2 / th) - d.gm1 * log_r(r2 / r);
  return q;
}

// The corrected entropy, one expression wherever it is formed (so any
// fused multiply-add is placed alike).
__device__ __forceinline__ real corr_s(real sv, const CorrDelta &q) { return sv + q.cv * q.ls; }

__global__ __launch_bounds__(kCorrThreads) void k_corr_apply(CorrArgs a) {
  __shared__ double tot[kCorrVals];
  const int k = blockIdx.y;
  if (threadIdx.x < kCorrVals) tot[threadIdx.x] = corr_total(a.partials, k, threadIdx.x);
  __syncthreads();
  const DomainArgs &d = a.doms[k];
  const CorrShift c = corr_shift(tot, a.n, a.conserve);
  real *st = a.state + a.offs[k];
  const long long P = d.plane;
  const long long base = (long long)k * a.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n;
       i += (long long)gridDim.x * blockDim.x) {
    const CorrDelta q = corr_delta(d, a.x + base, a.dl + base, a.sc, i, c);
    const long long o = state_off(d, i);
#pragma unroll
    for (int p = 0; p < kQ; ++p) st[p * P + o] += q.df[p];
    st[9 * P + o] = corr_s(st[9 * P + o], q);
  }
}

// Macroscopic fields of every domain of a batch in one launch: workgroup
// column y = domain, fields concatenated at foffs[k] (as k_moments per domain).
struct BatchFieldArgs {
  const DomainArgs *doms;
  const long long *offs, *foffs;
  const real *state;
  real *rho, *ux, *uy, *s, *theta;
};

__global__ __launch_bounds__(256) void k_batch_moments(BatchFieldArgs a) {
  const int k = blockIdx.y;
  const DomainArgs &d = a.doms[k];
  const long long n = (long long)d.nx * d.ny, P = d.plane;
  const real *st = a.state + a.offs[k];
  const long long fo = a.foffs[k];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const long long o = state_off(d, i);
    real F[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) F[q] = st[q * P + o];
    const real sv = st[9 * P + o];
    const NodeMoments m = node_moments(F, d);
    if (a.rho) a.rho[fo + i] = m.rho;
    if (a.ux) a.ux[fo + i] = m.jx / m.rho;
    if (a.uy) a.uy[fo + i] = m.jy / m.rho;
    if (a.s) a.s[fo + i] = sv + d.s_ref;
    if (a.theta) a.theta[fo + i] = node_theta(m.rho, sv, d);
  }
}

}  // namespace HLBM_NS
}  // namespace hlbm
