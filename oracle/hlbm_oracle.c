/*
 * FP64 CPU oracle of the D2Q9 hybrid lattice-Boltzmann step (HLBM).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against; nothing in the product links or calls it.
 * It shares no code, header, table or helper with the GPU path.
 *
 * It follows the HLBM algorithm of Sec. 3.5 (Algorithm 1) step by step, with
 * the formulas of Sec. 2 and Sec. 3:
 *   - lattice and weights: Sec. 2.1;
 *   - equilibrium as the Hermite expansion of Eq. (Equilibrium) with the
 *     coefficients of Eqs. (a0)-(a4) and the polynomials of Eqs. (H0)-(H4),
 *     restricted to the nine D2Q9 basis polynomials of Sec. 2.3;
 *   - correction term psi of Eq. (Psialgo) with E1 (Sec. 2.3, upwind scheme of
 *     Sec. 3.2) and E2 (Eq. E2 corr term, centred);
 *   - HRR reconstruction: Eq. (a1sigalgo), projection a1PR, finite-difference
 *     a1FD (Eq. a1FD), recursion to xxy, yyx, xxyy (Sec. 3.3);
 *   - collide-and-stream Eq. (streamalgo) with push streaming;
 *   - entropy update Eq. (sequaalgo): MUSCL/van Albada advection, centred
 *     Fourier term, viscous heat Eq. (viscous heat discret), explicit Euler;
 *   - closures p = rho c_s^2 theta (Eq. perfect gas), s = c_v ln(theta /
 *     rho^(gamma-1)) (Eq. Entropie expression), c_v, c_p of Sec. 2.4,
 *     mu = tau p (Sec. 2.4).
 * Lattice units: Dx = Dt = 1, c_s^2 = 1/3.
 *
 * Structure (deliberately unlike a fused kernel): ghost-padded arrays of depth
 * 2; one full-grid pass per algorithm stage; explicit per-population arrays
 * for f^eq, f^1 and psi; the equilibrium and off-equilibrium populations are
 * evaluated by the literal Hermite contraction over all index tuples.
 *
 * Readings of points the paper leaves open (each is listed with its reason in
 * the design notes): constant mu, local tau = mu / p; lambda = mu c_p / Pr;
 * sgn(0) = 0 in E1 (centred average); non-conservative MUSCL with node-sign
 * upwinding and the van Albada slope; sgn(u) in E1 is 0 inside a rounding
 * band |u| <= sgn_eps (the literal sign is discontinuous at u = 0 and turns
 * rounding noise into O(dGamma) jumps at wave fronts); 5-point Laplacian for the Fourier term;
 * boundaries per axis either periodic or zero-gradient (ghost = copy of the
 * nearest interior node state), or, along y, two isothermal moving walls.
 *
 * Walls (the paper's thermal Couette flow of Sec. 4.4 cites its wall
 * condition to an earlier paper without stating it; this is our own reading,
 * a regularised wet-node wall).  The wall rows y = 0 and y = ny - 1 are nodes
 * of the grid, H = ny - 1 apart, beyond which ghosts are zero-gradient.
 * After every step each wall node is rebuilt from its wall velocity
 * (U_wall, 0) and temperature theta_w:
 *   rho_w = sum of the populations with c_y = 0 + twice the sum of those that
 *           arrived from the interior (zero mass flux through the wall);
 *   F_w   = f^eq(rho_w, U_wall, 0, theta_w) + fbar^1[a1FD] with a1FD from the
 *           velocity gradient at the wall: zero along the wall, one-sided
 *           second order across it, (-3 u_0 + 4 u_1 - u_2) / 2 from the new
 *           velocities of the next two rows; psi is taken as zero there;
 *   s_w   = c_v ln(theta_w / rho_w^(gamma - 1)).
 * The collision at a wall node uses the projected stress alone (sigma = 1),
 * which recovers that a1FD.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9
#define GH 2 /* ghost depth = stencil radius */

static const int CXv[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CYv[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double Wv[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2v = 1.0 / 3.0;

typedef struct {
  int32_t nx, ny;
  int32_t bc_x, bc_y;   /* 0 periodic, 1 zero-gradient extrapolation; bc_y 2: walls */
  int32_t phi_mode;     /* 0: Phi from a1 (LBM), 1: Phi by finite differences */
  int32_t e1_centred;   /* ablation: 1 = centred E1 (original model) */
  int32_t e2_off;       /* ablation: 1 = no E2 term (original model) */
  int32_t feq_order;    /* 4 (present model) or 3 (original model) */
  double gamma, prandtl, mu, sigma;
  double sgn_eps;       /* |u| <= sgn_eps counts as sgn(u) = 0 in E1 (0: literal sign) */
  /* bc_y = 2: wall rows y = 0 and y = ny - 1 move along x with wall_ux_lo /
   * wall_ux_hi and are held at temperature wall_theta */
  double wall_ux_lo, wall_ux_hi, wall_theta;
} ora_params;

/* ------------------------------------------------------------------------- */
/* Hermite machinery: tensors over index tuples in {0 = x, 1 = y}^n           */
/* ------------------------------------------------------------------------- */

static double delta(int a, int b) { return a == b ? 1.0 : 0.0; }

/* Eqs. (H0)-(H4): Hermite polynomial H^(n)_{i, idx} for velocity c. */
static double hermite(const double c[2], int n, const int *k) {
  const double s = CS2v;
  switch (n) {
  case 0:
    return 1.0;
  case 1:
    return c[k[0]];
  case 2:
    return c[k[0]] * c[k[1]] - s * delta(k[0], k[1]);
  case 3:
    return c[k[0]] * c[k[1]] * c[k[2]] -
           s * (c[k[0]] * delta(k[1], k[2]) + c[k[1]] * delta(k[0], k[2]) +
                c[k[2]] * delta(k[0], k[1]));
  case 4: {
    int a = k[0], b = k[1], g = k[2], d = k[3];
    double t4 = c[a] * c[b] * c[g] * c[d];
    double t2 = c[a] * c[b] * delta(g, d) + c[a] * c[g] * delta(b, d) +
                c[a] * c[d] * delta(b, g) + c[b] * c[g] * delta(a, d) +
                c[b] * c[d] * delta(a, g) + c[g] * c[d] * delta(a, b);
    double t0 = delta(a, b) * delta(g, d) + delta(a, g) * delta(b, d) + delta(a, d) * delta(b, g);
    return t4 - s * t2 + s * s * t0;
  }
  }
  return 0.0;
}

/* Eqs. (a0)-(a4): equilibrium Hermite coefficient a^(n)_{idx}(rho, u, theta). */
static double aeq(int n, const int *k, double rho, const double u[2], double theta) {
  const double s = CS2v, t1 = theta - 1.0;
  switch (n) {
  case 0:
    return rho;
  case 1:
    return rho * u[k[0]];
  case 2:
    return rho * u[k[0]] * u[k[1]] + rho * s * t1 * delta(k[0], k[1]);
  case 3:
    return rho * u[k[0]] * u[k[1]] * u[k[2]] +
           rho * s * t1 *
               (u[k[0]] * delta(k[1], k[2]) + u[k[1]] * delta(k[0], k[2]) +
                u[k[2]] * delta(k[0], k[1]));
  case 4: {
    int a = k[0], b = k[1], g = k[2], d = k[3];
    double t4 = rho * u[a] * u[b] * u[g] * u[d];
    double t0 = rho * s * s * t1 * t1 *
                (delta(a, b) * delta(g, d) + delta(a, g) * delta(b, d) + delta(a, d) * delta(b, g));
    double t2 = rho * s * t1 *
                (u[a] * u[b] * delta(g, d) + u[a] * u[g] * delta(b, d) + u[a] * u[d] * delta(b, g) +
                 u[b] * u[g] * delta(a, d) + u[b] * u[d] * delta(a, g) + u[g] * u[d] * delta(a, b));
    return t4 + t0 + t2;
  }
  }
  return 0.0;
}

/* Sec. 2.3: a tuple is kept iff its multiset (#x, #y) is one of the nine D2Q9
 * basis polynomials 0, x, y, xx, xy, yy, xxy, yyx, xxyy.  Truncating the
 * expansion at order three (original model) drops xxyy. */
static int in_basis(int n, const int *k, int max_order) {
  int ny = 0;
  for (int j = 0; j < n; ++j) ny += k[j];
  int nxc = n - ny;
  if (n > max_order) return 0;
  return nxc <= 2 && ny <= 2;
}

static double factorial(int n) {
  double f = 1.0;
  for (int j = 2; j <= n; ++j) f *= j;
  return f;
}

/* Table of (i, n, tuple) -> H and kept flag; tuples enumerated in binary. */
static double HT[Q][5][16];
static int KEEP4[5][16], KEEP3[5][16];
static int tables_ready = 0;

static void tuple_of(int n, int code, int *k) {
  for (int j = 0; j < n; ++j) k[j] = (code >> (n - 1 - j)) & 1;
}

static void init_tables(void) {
  if (tables_ready) return;
  for (int i = 0; i < Q; ++i) {
    double c[2] = {(double)CXv[i], (double)CYv[i]};
    for (int n = 0; n <= 4; ++n)
      for (int code = 0; code < (1 << n); ++code) {
        int k[4];
        tuple_of(n, code, k);
        HT[i][n][code] = hermite(c, n, k);
      }
  }
  for (int n = 0; n <= 4; ++n)
    for (int code = 0; code < (1 << n); ++code) {
      int k[4];
      tuple_of(n, code, k);
      KEEP4[n][code] = in_basis(n, k, 4);
      KEEP3[n][code] = in_basis(n, k, 3);
    }
  tables_ready = 1;
}

/* Eq. (Equilibrium): f^eq_i = w_i sum_n 1/(n! c_s^2n) a^(n) : H^(n)_i. */
static void feq_point(double rho, double ux, double uy, double theta, int order, double out[Q]) {
  init_tables();
  const double u[2] = {ux, uy};
  double A[5][16];
  for (int n = 0; n <= 4; ++n)
    for (int code = 0; code < (1 << n); ++code) {
      int k[4];
      tuple_of(n, code, k);
      A[n][code] = aeq(n, k, rho, u, theta);
    }
  for (int i = 0; i < Q; ++i) {
    double sum = 0.0;
    for (int n = 0; n <= 4; ++n) {
      double part = 0.0;
      for (int code = 0; code < (1 << n); ++code) {
        int keep = order >= 4 ? KEEP4[n][code] : KEEP3[n][code];
        if (keep) part += A[n][code] * HT[i][n][code];
      }
      sum += part / (factorial(n) * pow(CS2v, n));
    }
    out[i] = Wv[i] * sum;
  }
}

/* Off-equilibrium Hermite coefficient of a kept tuple, from its multiset. */
static double a1_of_tuple(int n, const int *k, const double a1[6]) {
  int ny = 0;
  for (int j = 0; j < n; ++j) ny += k[j];
  int nxc = n - ny;
  if (nxc == 2 && ny == 0) return a1[0]; /* xx   */
  if (nxc == 1 && ny == 1) return a1[1]; /* xy   */
  if (nxc == 0 && ny == 2) return a1[2]; /* yy   */
  if (nxc == 2 && ny == 1) return a1[3]; /* xxy  */
  if (nxc == 1 && ny == 2) return a1[4]; /* yyx  */
  if (nxc == 2 && ny == 2) return a1[5]; /* xxyy */
  return 0.0;
}

/* Sec. 3.3 recursion: higher off-equilibrium moments from a1_{alpha beta}. */
static void a1_recursion(double a1xx, double a1xy, double a1yy, double ux, double uy, double theta,
                         double out[6]) {
  const double c = CS2v * (theta - 1.0);
  double axxy = uy * a1xx + 2.0 * ux * a1xy;
  double ayyx = ux * a1yy + 2.0 * uy * a1xy;
  double axxyy = 2.0 * (ux * ayyx + uy * axxy) + (c - ux * ux) * a1yy + (c - uy * uy) * a1xx -
                 4.0 * ux * uy * a1xy;
  out[0] = a1xx;
  out[1] = a1xy;
  out[2] = a1yy;
  out[3] = axxy;
  out[4] = ayyx;
  out[5] = axxyy;
}

/* Sec. 3.3: fbar^1_i = w_i sum_{n>=2} 1/(n! c_s^2n) a1^(n) : H^(n)_i. */
static void f1_point(const double a1[6], int order, double out[Q]) {
  init_tables();
  for (int i = 0; i < Q; ++i) {
    double sum = 0.0;
    for (int n = 2; n <= 4; ++n) {
      double part = 0.0;
      for (int code = 0; code < (1 << n); ++code) {
        int keep = order >= 4 ? KEEP4[n][code] : KEEP3[n][code];
        if (!keep) continue;
        int k[4];
        tuple_of(n, code, k);
        part += a1_of_tuple(n, k, a1) * HT[i][n][code];
      }
      sum += part / (factorial(n) * pow(CS2v, n));
    }
    out[i] = Wv[i] * sum;
  }
}

/* Eq. (Psialgo): psi_i = w_i H_{i,ab} E_ab / (2 c_s^4), E diagonal. */
static void psi_point(double Exx, double Eyy, double out[Q]) {
  init_tables();
  for (int i = 0; i < Q; ++i) {
    double sum = 0.0;
    for (int code = 0; code < 4; ++code) {
      int k[2];
      tuple_of(2, code, k);
      double E = (k[0] == k[1]) ? (k[0] == 0 ? Exx : Eyy) : 0.0;
      sum += HT[i][2][code] * E;
    }
    out[i] = Wv[i] * sum / (2.0 * CS2v * CS2v);
  }
}

/* ------------------------------------------------------------------------- */
/* Grid state                                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
  ora_params p;
  int px, py;
  size_t np;
  double cv, cp, lambda;
  double *F[Q], *Fn[Q], *s, *sn;
  double *rho, *ux, *uy, *th, *pr, *tau, *taub;
  double *dxux, *dyux, *dxuy, *dyuy;
  double *gx, *gy, *Exx, *Eyy;
  double *a1xx, *a1xy, *a1yy;
  double *feq[Q], *f1[Q], *psi[Q], *fst[Q];
  double *phi;
  long steps;
} ora_state;

static inline size_t IX(const ora_state *S, int X, int Y) { return (size_t)Y * S->px + X; }

static int map_index(int v, int n, int bc) {
  if (bc == 0) {
    int r = v % n;
    return r < 0 ? r + n : r;
  }
  return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

static double *alloc_field(size_t n) { return (double *)calloc(n, sizeof(double)); }

void *ora_create(const ora_params *p) {
  if (!p || p->nx < 1 || p->ny < 1) return NULL;
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 2) return NULL;
  if (p->bc_y == 2 && (p->ny < 4 || !(p->wall_theta > 0.0))) return NULL;
  init_tables();
  ora_state *S = (ora_state *)calloc(1, sizeof(ora_state));
  S->p = *p;
  if (S->p.feq_order != 3) S->p.feq_order = 4;
  S->px = p->nx + 2 * GH;
  S->py = p->ny + 2 * GH;
  S->np = (size_t)S->px * S->py;
  S->cv = CS2v / (p->gamma - 1.0);
  S->cp = p->gamma * CS2v / (p->gamma - 1.0);
  S->lambda = p->mu * S->cp / p->prandtl;
  for (int i = 0; i < Q; ++i) {
    S->F[i] = alloc_field(S->np);
    S->Fn[i] = alloc_field(S->np);
    S->feq[i] = alloc_field(S->np);
    S->f1[i] = alloc_field(S->np);
    S->psi[i] = alloc_field(S->np);
    S->fst[i] = alloc_field(S->np);
  }
  double **fl[] = {&S->s,    &S->sn,   &S->rho,  &S->ux,   &S->uy,   &S->th,   &S->pr,
                   &S->tau,  &S->taub, &S->dxux, &S->dyux, &S->dxuy, &S->dyuy, &S->gx,
                   &S->gy,   &S->Exx,  &S->Eyy,  &S->a1xx, &S->a1xy, &S->a1yy, &S->phi};
  for (size_t j = 0; j < sizeof(fl) / sizeof(fl[0]); ++j) *fl[j] = alloc_field(S->np);
  return S;
}

void ora_destroy(void *h) {
  ora_state *S = (ora_state *)h;
  if (!S) return;
  for (int i = 0; i < Q; ++i) {
    free(S->F[i]);
    free(S->Fn[i]);
    free(S->feq[i]);
    free(S->f1[i]);
    free(S->psi[i]);
    free(S->fst[i]);
  }
  double *fl[] = {S->s,    S->sn,   S->rho,  S->ux,   S->uy,   S->th,   S->pr,
                  S->tau,  S->taub, S->dxux, S->dyux, S->dxuy, S->dyuy, S->gx,
                  S->gy,   S->Exx,  S->Eyy,  S->a1xx, S->a1xy, S->a1yy, S->phi};
  for (size_t j = 0; j < sizeof(fl) / sizeof(fl[0]); ++j) free(fl[j]);
  free(S);
}

/* Ghost layers: copy of the mapped interior node (periodic wrap or clamp). */
static void fill_ghosts(ora_state *S, double **arrs, int count) {
  const int nx = S->p.nx, ny = S->p.ny;
#pragma omp parallel for schedule(static)
  for (int Y = 0; Y < S->py; ++Y) {
    for (int X = 0; X < S->px; ++X) {
      int x = X - GH, y = Y - GH;
      if (x >= 0 && x < nx && y >= 0 && y < ny) continue;
      int sx = map_index(x, nx, S->p.bc_x) + GH;
      int sy = map_index(y, ny, S->p.bc_y) + GH;
      for (int a = 0; a < count; ++a) arrs[a][IX(S, X, Y)] = arrs[a][IX(S, sx, sy)];
    }
  }
}

static void fill_state_ghosts(ora_state *S) {
  double *arrs[Q + 1];
  for (int i = 0; i < Q; ++i) arrs[i] = S->F[i];
  arrs[Q] = S->s;
  fill_ghosts(S, arrs, Q + 1);
}

/* Eq. (Entropie expression) inverted: theta = rho^(gamma-1) exp(s / c_v). */
static double theta_of(const ora_state *S, double rho, double s) {
  return pow(rho, S->p.gamma - 1.0) * exp(s / S->cv);
}

/* Node-local thermodynamics from (rho, u, s): theta, p, tau = mu / p, taubar. */
static void thermo_pass(ora_state *S, int ring) {
  const int lo = GH - ring, hix = GH + S->p.nx + ring, hiy = GH + S->p.ny + ring;
#pragma omp parallel for schedule(static)
  for (int Y = lo; Y < hiy; ++Y)
    for (int X = lo; X < hix; ++X) {
      size_t k = IX(S, X, Y);
      double th = theta_of(S, S->rho[k], S->s[k]);
      S->th[k] = th;
      S->pr[k] = S->rho[k] * CS2v * th;         /* Eq. (perfect gas) */
      S->tau[k] = S->p.mu / S->pr[k];           /* mu = tau p        */
      S->taub[k] = S->tau[k] + 0.5;             /* taubar = tau + Dt/2 */
    }
}

/* Eqs. (rhoalgo), (ualgo): zeroth and first moments of the populations. */
static void moments_pass(ora_state *S) {
#pragma omp parallel for schedule(static)
  for (int Y = 0; Y < S->py; ++Y)
    for (int X = 0; X < S->px; ++X) {
      size_t k = IX(S, X, Y);
      double r = 0.0, jx = 0.0, jy = 0.0;
      for (int i = 0; i < Q; ++i) {
        r += S->F[i][k];
        jx += CXv[i] * S->F[i][k];
        jy += CYv[i] * S->F[i][k];
      }
      S->rho[k] = r;
      S->ux[k] = jx / r;
      S->uy[k] = jy / r;
    }
}

/* Centred velocity gradients, Gamma, E1 (upwind) and E2 (centred) on the
 * interior plus one ghost ring (Sec. 3.2). */
static void gradient_pass(ora_state *S) {
  const int lo = GH - 1, hix = GH + S->p.nx + 1, hiy = GH + S->p.ny + 1;
  const double D = 2.0;
  /* Gamma = rho u_a (1 - theta - u_a^2) = -a^eq_aaa, needed at radius 2. */
#pragma omp parallel for schedule(static)
  for (int Y = 0; Y < S->py; ++Y)
    for (int X = 0; X < S->px; ++X) {
      size_t k = IX(S, X, Y);
      double u = S->ux[k], v = S->uy[k];
      S->gx[k] = S->rho[k] * u * (1.0 - S->th[k] - u * u);
      S->gy[k] = S->rho[k] * v * (1.0 - S->th[k] - v * v);
    }
#pragma omp parallel for schedule(static)
  for (int Y = lo; Y < hiy; ++Y)
    for (int X = lo; X < hix; ++X) {
      size_t k = IX(S, X, Y);
      size_t e = IX(S, X + 1, Y), w = IX(S, X - 1, Y), n = IX(S, X, Y + 1), so = IX(S, X, Y - 1);
      S->dxux[k] = 0.5 * (S->ux[e] - S->ux[w]);
      S->dyux[k] = 0.5 * (S->ux[n] - S->ux[so]);
      S->dxuy[k] = 0.5 * (S->uy[e] - S->uy[w]);
      S->dyuy[k] = 0.5 * (S->uy[n] - S->uy[so]);
      double div = S->dxux[k] + S->dyuy[k];
      /* E1_xx: [1+sgn(ux)]/2 (G_i - G_{i-1}) + [1-sgn(ux)]/2 (G_{i+1} - G_i);
       * a velocity within the rounding band |u| <= sgn_eps has sign 0. */
      const double eps = S->p.sgn_eps;
      double sx = (S->ux[k] > eps) ? 1.0 : ((S->ux[k] < -eps) ? -1.0 : 0.0);
      double sy = (S->uy[k] > eps) ? 1.0 : ((S->uy[k] < -eps) ? -1.0 : 0.0);
      if (S->p.e1_centred) {
        sx = 0.0;
        sy = 0.0;
      }
      double e1x = 0.5 * (1.0 + sx) * (S->gx[k] - S->gx[w]) + 0.5 * (1.0 - sx) * (S->gx[e] - S->gx[k]);
      double e1y = 0.5 * (1.0 + sy) * (S->gy[k] - S->gy[so]) + 0.5 * (1.0 - sy) * (S->gy[n] - S->gy[k]);
      /* Eq. (E2 corr term): p ((D+2)/D - gamma) div u */
      double e2 = S->p.e2_off ? 0.0 : S->pr[k] * ((D + 2.0) / D - S->p.gamma) * div;
      S->Exx[k] = e1x + e2;
      S->Eyy[k] = e1y + e2;
    }
}

/* f^eq, psi, HRR off-equilibrium and post-collision populations on the
 * interior plus one ghost ring (Sec. 3.3, Eq. streamalgo). */
static void collide_pass(ora_state *S) {
  const int lo = GH - 1, hix = GH + S->p.nx + 1, hiy = GH + S->p.ny + 1;
  const int order = S->p.feq_order;
  const double sig = S->p.sigma;
#pragma omp parallel for schedule(static)
  for (int Y = lo; Y < hiy; ++Y)
    for (int X = lo; X < hix; ++X) {
      size_t k = IX(S, X, Y);
      double fe[Q], ps[Q];
      feq_point(S->rho[k], S->ux[k], S->uy[k], S->th[k], order, fe);
      psi_point(S->Exx[k], S->Eyy[k], ps);
      /* a1PR_ab = sum_i H_i,ab (fbar_i - feq_i + psi_i / 2) */
      double pr[3] = {0.0, 0.0, 0.0};
      for (int i = 0; i < Q; ++i) {
        double g = S->F[i][k] - fe[i] + 0.5 * ps[i];
        pr[0] += HT[i][2][0] * g; /* (x,x) */
        pr[1] += HT[i][2][1] * g; /* (x,y) */
        pr[2] += HT[i][2][3] * g; /* (y,y) */
      }
      /* a1FD_ab = -(taubar/tau) mu (d_b u_a + d_a u_b - (2/D) div delta_ab);
       * with mu = tau p the prefactor is taubar p (finite for mu = 0). */
      double tp = S->taub[k] * S->pr[k];
      double div = S->dxux[k] + S->dyuy[k];
      double fd[3];
      fd[0] = -tp * (2.0 * S->dxux[k] - div);
      fd[1] = -tp * (S->dyux[k] + S->dxuy[k]);
      fd[2] = -tp * (2.0 * S->dyuy[k] - div);
      /* wall nodes: projection only (their populations carry the wall stress) */
      const int wall_row = S->p.bc_y == 2 && (Y == GH || Y == GH + S->p.ny - 1);
      const double sg = wall_row ? 1.0 : sig;
      double a1[3];
      for (int j = 0; j < 3; ++j) a1[j] = sg * pr[j] + (1.0 - sg) * fd[j];
      S->a1xx[k] = a1[0];
      S->a1xy[k] = a1[1];
      S->a1yy[k] = a1[2];
      double a1full[6], f1v[Q];
      a1_recursion(a1[0], a1[1], a1[2], S->ux[k], S->uy[k], S->th[k], a1full);
      f1_point(a1full, order, f1v);
      double om = 1.0 - 1.0 / S->taub[k];
      for (int i = 0; i < Q; ++i) {
        S->feq[i][k] = fe[i];
        S->psi[i][k] = ps[i];
        S->f1[i][k] = f1v[i];
        S->fst[i][k] = fe[i] + om * f1v[i] + 0.5 * ps[i];
      }
    }
}

/* Push streaming: F'_i(x + c_i) = f*_i(x) for every target inside the grid. */
static void stream_pass(ora_state *S) {
  const int nx = S->p.nx, ny = S->p.ny;
#pragma omp parallel for schedule(static)
  for (int Y = GH - 1; Y < GH + ny + 1; ++Y)
    for (int X = GH - 1; X < GH + nx + 1; ++X) {
      size_t k = IX(S, X, Y);
      for (int i = 0; i < Q; ++i) {
        int tx = X + CXv[i], ty = Y + CYv[i];
        if (tx < GH || tx >= GH + nx || ty < GH || ty >= GH + ny) continue;
        S->Fn[i][IX(S, tx, ty)] = S->fst[i][k];
      }
    }
}

/* van Albada limited slope of (a, b) = backward and forward differences:
 * phi(r) b with phi(r) = (r^2 + r)/(r^2 + 1), r = a / b, zero for r <= 0. */
static double van_albada(double a, double b) {
  if (a * b <= 0.0) return 0.0;
  double r = a / b;
  return (r * r + r) / (r * r + 1.0) * b;
}

/* Upwind MUSCL derivative of s along one axis at node k (stride st). */
static double muscl_derivative(const double *s, size_t k, long st, double vel) {
  if (vel == 0.0) return 0.0;
  double sm2 = s[k - 2 * st], sm1 = s[k - st], s0 = s[k], sp1 = s[k + st], sp2 = s[k + 2 * st];
  if (vel > 0.0) {
    double dl = van_albada(s0 - sm1, sp1 - s0);    /* slope at i   */
    double dlm = van_albada(sm1 - sm2, s0 - sm1);  /* slope at i-1 */
    double face_r = s0 + 0.5 * dl;                 /* left state at i+1/2 */
    double face_l = sm1 + 0.5 * dlm;               /* left state at i-1/2 */
    return face_r - face_l;
  } else {
    double dl = van_albada(s0 - sm1, sp1 - s0);    /* slope at i   */
    double dlp = van_albada(sp1 - s0, sp2 - sp1);  /* slope at i+1 */
    double face_r = sp1 - 0.5 * dlp;               /* right state at i+1/2 */
    double face_l = s0 - 0.5 * dl;                 /* right state at i-1/2 */
    return face_r - face_l;
  }
}

/* Eq. (sequaalgo) with explicit Euler, evaluated with level-n fields. */
static void entropy_pass(ora_state *S) {
  const int nx = S->p.nx, ny = S->p.ny;
  const long sy = S->px;
#pragma omp parallel for schedule(static)
  for (int Y = GH; Y < GH + ny; ++Y)
    for (int X = GH; X < GH + nx; ++X) {
      size_t k = IX(S, X, Y);
      double adv = S->ux[k] * muscl_derivative(S->s, k, 1, S->ux[k]) +
                   S->uy[k] * muscl_derivative(S->s, k, sy, S->uy[k]);
      double lap = S->th[k + 1] + S->th[k - 1] + S->th[k + sy] + S->th[k - sy] - 4.0 * S->th[k];
      double four = S->lambda * lap;
      double phi;
      if (S->p.phi_mode == 0) {
        /* Phi = -(tau / taubar) a1_ab d_b u_a */
        double contr = S->a1xx[k] * S->dxux[k] + S->a1xy[k] * S->dyux[k] +
                       S->a1xy[k] * S->dxuy[k] + S->a1yy[k] * S->dyuy[k];
        phi = -(S->tau[k] / S->taub[k]) * contr;
      } else {
        /* Eq. (viscous heat): mu (d_b u_a + d_a u_b - (2/D) div delta) d_b u_a */
        double g[2][2] = {{S->dxux[k], S->dyux[k]}, {S->dxuy[k], S->dyuy[k]}}; /* g[a][b] = d_b u_a */
        double div = g[0][0] + g[1][1];
        double sum = 0.0;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            sum += (g[a][b] + g[b][a] - (a == b ? div : 0.0)) * g[a][b];
        phi = S->p.mu * sum;
      }
      S->phi[k] = phi;
      S->sn[k] = S->s[k] - adv + (four + phi) / (S->rho[k] * S->th[k]);
    }
}

static void swap_buffers(ora_state *S) {
  for (int i = 0; i < Q; ++i) {
    double *t = S->F[i];
    S->F[i] = S->Fn[i];
    S->Fn[i] = t;
  }
  double *t = S->s;
  S->s = S->sn;
  S->sn = t;
}

/* Derived fields of the current state (steps 6, 8-11 of the algorithm are the
 * opening passes of the next step). */
static void derive(ora_state *S) {
  fill_state_ghosts(S);
  moments_pass(S);
  thermo_pass(S, GH);
  gradient_pass(S);
  collide_pass(S);
}

/* Velocity of node (X, Y) from its populations. */
static void node_velocity(const ora_state *S, size_t k, double *ux, double *uy) {
  double r = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < Q; ++i) {
    r += S->F[i][k];
    jx += CXv[i] * S->F[i][k];
    jy += CYv[i] * S->F[i][k];
  }
  *ux = jx / r;
  *uy = jy / r;
}

/* Rebuild the two wall rows (see the header).  side 0: y = 0, whose
 * populations with c_y = -1 came from the interior; side 1: y = ny - 1, c_y
 * = +1.  Reads only rows 1, 2 and ny - 2, ny - 3 besides the wall rows. */
static void wall_pass(ora_state *S) {
  const int nx = S->p.nx, ny = S->p.ny, order = S->p.feq_order;
  const double thw = S->p.wall_theta;
  for (int X = GH; X < GH + nx; ++X) {
    double Fnew[2][Q], snew[2];
    for (int side = 0; side < 2; ++side) {
      const int Yw = side == 0 ? GH : GH + ny - 1;
      const int dir = side == 0 ? 1 : -1;              /* towards the interior */
      const double U = side == 0 ? S->p.wall_ux_lo : S->p.wall_ux_hi;
      const size_t kw = IX(S, X, Yw);
      double rho = 0.0;
      for (int i = 0; i < Q; ++i) {
        if (CYv[i] == 0) rho += S->F[i][kw];
        else if (CYv[i] == -dir) rho += 2.0 * S->F[i][kw];  /* arrived from the interior */
      }
      double u1x, u1y, u2x, u2y;
      node_velocity(S, IX(S, X, Yw + dir), &u1x, &u1y);
      node_velocity(S, IX(S, X, Yw + 2 * dir), &u2x, &u2y);
      /* d/dy, one-sided second order; the wall-normal velocity is zero */
      const double dyux = dir * (-3.0 * U + 4.0 * u1x - u2x) / 2.0;
      const double dyuy = dir * (4.0 * u1y - u2y) / 2.0;
      const double pw = rho * CS2v * thw;
      const double tp = (S->p.mu / pw + 0.5) * pw;      /* taubar p */
      const double div = dyuy;
      const double axx = -tp * (0.0 - div), axy = -tp * dyux, ayy = -tp * (2.0 * dyuy - div);
      double fe[Q], f1v[Q], a1full[6];
      feq_point(rho, U, 0.0, thw, order, fe);
      a1_recursion(axx, axy, ayy, U, 0.0, thw, a1full);
      f1_point(a1full, order, f1v);
      for (int i = 0; i < Q; ++i) Fnew[side][i] = fe[i] + f1v[i];
      snew[side] = S->cv * log(thw / pow(rho, S->p.gamma - 1.0));
    }
    for (int side = 0; side < 2; ++side) {
      const size_t kw = IX(S, X, side == 0 ? GH : GH + ny - 1);
      for (int i = 0; i < Q; ++i) S->F[i][kw] = Fnew[side][i];
      S->s[kw] = snew[side];
    }
  }
}

void ora_step(void *h, int nsteps) {
  ora_state *S = (ora_state *)h;
  for (int n = 0; n < nsteps; ++n) {
    derive(S);
    stream_pass(S);
    entropy_pass(S);
    swap_buffers(S);
    if (S->p.bc_y == 2) wall_pass(S);
    S->steps++;
  }
}

/* Initialisation (Algorithm, steps 1-4): F^0 = f^eq + fbar^1[a1FD] - psi / 2
 * from (rho, u, s); the first step then sees a1PR = a1FD for any sigma. */
void ora_init(void *h, const double *rho, const double *ux, const double *uy, const double *s) {
  ora_state *S = (ora_state *)h;
  const int nx = S->p.nx, ny = S->p.ny;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = IX(S, x + GH, y + GH), j = (size_t)y * nx + x;
      S->rho[k] = rho[j];
      S->ux[k] = ux[j];
      S->uy[k] = uy[j];
      S->s[k] = s[j];
    }
  double *arrs[4] = {S->rho, S->ux, S->uy, S->s};
  fill_ghosts(S, arrs, 4);
  thermo_pass(S, GH);
  gradient_pass(S);
  const int order = S->p.feq_order;
  for (int Y = GH; Y < GH + ny; ++Y)
    for (int X = GH; X < GH + nx; ++X) {
      size_t k = IX(S, X, Y);
      double fe[Q], ps[Q], f1v[Q], a1full[6];
      feq_point(S->rho[k], S->ux[k], S->uy[k], S->th[k], order, fe);
      psi_point(S->Exx[k], S->Eyy[k], ps);
      double tp = S->taub[k] * S->pr[k];
      double div = S->dxux[k] + S->dyuy[k];
      double fxx = -tp * (2.0 * S->dxux[k] - div);
      double fxy = -tp * (S->dyux[k] + S->dxuy[k]);
      double fyy = -tp * (2.0 * S->dyuy[k] - div);
      a1_recursion(fxx, fxy, fyy, S->ux[k], S->uy[k], S->th[k], a1full);
      f1_point(a1full, order, f1v);
      for (int i = 0; i < Q; ++i) S->F[i][k] = fe[i] + f1v[i] - 0.5 * ps[i];
    }
  if (S->p.bc_y == 2) wall_pass(S);
  S->steps = 0;
}

/* State access ------------------------------------------------------------ */

void ora_get_state(void *h, double *F9, double *s) {
  ora_state *S = (ora_state *)h;
  const int nx = S->p.nx, ny = S->p.ny;
  size_t n = (size_t)nx * ny;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = IX(S, x + GH, y + GH), j = (size_t)y * nx + x;
      for (int i = 0; i < Q; ++i) F9[i * n + j] = S->F[i][k];
      s[j] = S->s[k];
    }
}

void ora_set_state(void *h, const double *F9, const double *s) {
  ora_state *S = (ora_state *)h;
  const int nx = S->p.nx, ny = S->p.ny;
  size_t n = (size_t)nx * ny;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = IX(S, x + GH, y + GH), j = (size_t)y * nx + x;
      for (int i = 0; i < Q; ++i) S->F[i][k] = F9[i * n + j];
      S->s[k] = s[j];
    }
}

/* Macroscopic fields of the current state: rho, u, s and theta. */
void ora_moments(void *h, double *rho, double *ux, double *uy, double *s, double *theta) {
  ora_state *S = (ora_state *)h;
  fill_state_ghosts(S);
  moments_pass(S);
  thermo_pass(S, 0);
  const int nx = S->p.nx, ny = S->p.ny;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = IX(S, x + GH, y + GH), j = (size_t)y * nx + x;
      if (rho) rho[j] = S->rho[k];
      if (ux) ux[j] = S->ux[k];
      if (uy) uy[j] = S->uy[k];
      if (s) s[j] = S->s[k];
      if (theta) theta[j] = S->th[k];
    }
}

/* Named derived field of the current state (after the opening passes of a
 * step; Phi is the value used by the last completed step). */
int ora_field(void *h, const char *name, double *out) {
  ora_state *S = (ora_state *)h;
  derive(S);
  const double *src = NULL;
  if (!strcmp(name, "a1xx")) src = S->a1xx;
  else if (!strcmp(name, "a1xy")) src = S->a1xy;
  else if (!strcmp(name, "a1yy")) src = S->a1yy;
  else if (!strcmp(name, "Exx")) src = S->Exx;
  else if (!strcmp(name, "Eyy")) src = S->Eyy;
  else if (!strcmp(name, "dxux")) src = S->dxux;
  else if (!strcmp(name, "dyux")) src = S->dyux;
  else if (!strcmp(name, "dxuy")) src = S->dxuy;
  else if (!strcmp(name, "dyuy")) src = S->dyuy;
  else if (!strcmp(name, "theta")) src = S->th;
  else if (!strcmp(name, "p")) src = S->pr;
  else if (!strcmp(name, "phi")) src = S->phi;
  else if (!strcmp(name, "tau")) src = S->tau;
  if (!src) return -1;
  const int nx = S->p.nx, ny = S->p.ny;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) out[(size_t)y * nx + x] = src[IX(S, x + GH, y + GH)];
  return 0;
}

/* Conservation totals: mass, x and y momentum, total energy
 * sum(rho c_v theta + rho |u|^2 / 2). */
void ora_totals(void *h, double out[4]) {
  ora_state *S = (ora_state *)h;
  fill_state_ghosts(S);
  moments_pass(S);
  thermo_pass(S, 0);
  double m = 0, px = 0, py = 0, e = 0;
  for (int Y = GH; Y < GH + S->p.ny; ++Y)
    for (int X = GH; X < GH + S->p.nx; ++X) {
      size_t k = IX(S, X, Y);
      double r = S->rho[k], u = S->ux[k], v = S->uy[k];
      m += r;
      px += r * u;
      py += r * v;
      e += r * S->cv * S->th[k] + 0.5 * r * (u * u + v * v);
    }
  out[0] = m;
  out[1] = px;
  out[2] = py;
  out[3] = e;
}

long ora_steps(void *h) { return ((ora_state *)h)->steps; }

/* Point functions exported for the identity checks ----------------------- */

void ora_feq(double rho, double ux, double uy, double theta, int order, double *out) {
  feq_point(rho, ux, uy, theta, order, out);
}

void ora_f1(double a1xx, double a1xy, double a1yy, double ux, double uy, double theta, int order,
            double *out) {
  double a1full[6];
  a1_recursion(a1xx, a1xy, a1yy, ux, uy, theta, a1full);
  f1_point(a1full, order, out);
}

void ora_f1_raw(const double *a1six, int order, double *out) { f1_point(a1six, order, out); }

void ora_psi(double Exx, double Eyy, double *out) { psi_point(Exx, Eyy, out); }

double ora_hermite(int i, int n, const int *k) {
  double c[2] = {(double)CXv[i], (double)CYv[i]};
  return hermite(c, n, k);
}

double ora_van_albada(double a, double b) { return van_albada(a, b); }

/* Eq. (Entropie expression): s = c_v ln(theta / rho^(gamma - 1)). */
void ora_entropy(const double *rho, const double *theta, double gamma, long n, double *s) {
  double cv = CS2v / (gamma - 1.0);
  for (long j = 0; j < n; ++j) s[j] = cv * log(theta[j] / pow(rho[j], gamma - 1.0));
}

/* Threads of the OpenMP passes: n > 0 sets the count for later calls; the
 * return value is the count in effect (1 without OpenMP). */
int ora_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}
