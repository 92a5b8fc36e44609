/*
 * hlbm.h -- C ABI of the MI355X (gfx950) hybrid lattice-Boltzmann library.
 *
 * One time step of the D2Q9 hybrid LBM of Renard, Feng, Boussuge and Sagaut
 * (arXiv 2002.03644): regularised (HRR) collision with the lattice-closure
 * correction psi (upwind E1 plus the polyatomic E2, Sec. 3.2), the recursive
 * off-equilibrium reconstruction (Sec. 3.3), streaming (Sec. 3.1), and the
 * finite-volume entropy update with the viscous heat production from the
 * regularised stress (Sec. 3.4), closed by p = rho c_s^2 theta and
 * s = c_v ln(theta / rho^(gamma-1)) (Sec. 2.1, 2.4).  The step order follows
 * the algorithm of Sec. 3.5.  Lattice units: Dx = Dt = 1, c_s^2 = 1/3.
 *
 * Conventions for every entry point
 *  - Fields are row-major [ny][nx] arrays, x fastest, contiguous; populations
 *    are nine such planes [9][ny][nx] in the lattice order
 *    c_x = {0,1,0,-1,0,1,-1,-1,1}, c_y = {0,0,1,0,-1,1,1,-1,-1}.
 *  - Array pointers are DEVICE pointers unless the name says host_.  Their
 *    element type is the handle's dtype (double for HLBM_F64, float for
 *    HLBM_F32).
 *  - The caller owns every device buffer, including the workspace; the library
 *    never allocates device memory.  The library owns only its small host
 *    handle, released by the matching destroy call.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is the
 *    default stream) and is asynchronous unless stated otherwise.
 *  - Errors are negative return codes (hlbm_status_code); nothing throws across the
 *    ABI.  A HIP launch failure is reported as HLBM_EHIP.
 *  - Calls on one handle must not overlap in time from several host threads.
 */
#ifndef HLBM_H
#define HLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *hlbm_stream_t; /* a hipStream_t */

typedef enum {
  HLBM_OK = 0,
  HLBM_WARN_CFL = 1,     /* init succeeded, but the largest local CFL number
                            (|u| + sqrt(gamma c_s^2 theta), Sec. 3.5) is >= 1 */
  HLBM_EINVAL = -1,      /* invalid parameter, size or pointer */
  HLBM_EWORKSPACE = -2,  /* workspace missing or smaller than required */
  HLBM_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
  HLBM_EDIVERGED = -4,   /* non-finite value, rho <= 0 or theta <= 0 found */
  HLBM_ENOMEM = -5       /* host allocation of the handle failed */
} hlbm_status_code;

typedef enum { HLBM_BC_PERIODIC = 0, HLBM_BC_EXTRAPOLATE = 1, HLBM_BC_WALL = 2 } hlbm_bc;
typedef enum { HLBM_F64 = 0, HLBM_F32 = 1 } hlbm_dtype;
typedef enum { HLBM_PHI_LBM = 0, HLBM_PHI_FD = 1 } hlbm_phi;

/* Parameters of one domain.  A zero-initialised struct plus nx, ny, gamma,
 * prandtl and the reference state selects the present model. */
typedef struct {
  int32_t nx, ny;       /* grid size, >= 1 each, 9 * nx * ny < 2^31; with rows padded
                           to pitch = nx rounded up to 64, also pitch * ny < 2^31
                           and pitch * ny * element size < 2^32 (the step
                           addresses a plane with 32-bit byte offsets) */
  int32_t bc_x, bc_y;   /* hlbm_bc on both sides of that axis: periodic wrap,
                           or zero-gradient extrapolation (the neighbour index
                           is clamped into the grid, so ghost nodes carry the
                           full state of the nearest boundary node); bc_y
                           alone may also be HLBM_BC_WALL: the rows y = 0 and
                           y = ny - 1 are isothermal walls moving along x
                           (ny >= 4; see hlbm_step), ghosts beyond them clamp */
  int32_t dtype;        /* hlbm_dtype of every array passed in or out */
  int32_t phi_mode;     /* viscous heat Phi: HLBM_PHI_LBM = -(tau/taubar) a1 : grad u
                           (Eq. viscous heat discret), HLBM_PHI_FD = finite
                           differences (Eq. viscous heat; for discontinuities) */
  int32_t e1_centred;   /* 0: upwind E1 of Sec. 3.2 (present model);
                           1: centred E1 (original-model ablation) */
  int32_t e2_off;       /* 0: with the polyatomic E2 term (present model);
                           1: without it (original-model ablation) */
  int32_t tile_w;       /* tile width in columns (64, 128, 192 or 256; the workgroup has
                           tile_w + 64 lanes, the extra wave holds the halo; 120, 184, 248
                           too with steps_per_launch = 2, whose workgroup is tile_w + 8
                           lanes rounded up to whole waves), 0 = auto */
  int32_t tile_h;       /* output rows per workgroup strip (>= 1), 0 = auto;
                           hlbm_launch_shape reports what a step will use */
  double gamma;         /* heat-capacity ratio, > 1 */
  double prandtl;       /* Prandtl number, > 0; lambda = mu c_p / Pr */
  double mu;            /* dynamic viscosity, >= 0; local tau = mu / p */
  double sigma;         /* HRR blend in [0, 1] (Eq. a1sigalgo) */
  double rho_ref;       /* HLBM_F32 storage reference density, > 0 */
  double theta_ref;     /* HLBM_F32 storage reference temperature, > 0 */
  double sgn_eps;       /* >= 0: the upwind E1 of Sec. 3.2 takes sgn(u) = 0 (centred
                           difference) for |u| <= sgn_eps.  0 is the literal sign,
                           which is discontinuous at u = 0; 1e-12 keeps
                           rounding-level velocities from flipping the stencil */
  double wall_ux_lo;    /* bc_y = HLBM_BC_WALL: x velocity of the wall row y = 0 */
  double wall_ux_hi;    /* bc_y = HLBM_BC_WALL: x velocity of the wall row y = ny - 1 */
  double wall_theta;    /* bc_y = HLBM_BC_WALL: temperature of both walls, > 0 */
  int32_t precise_theta; /* 0: theta = theta_ref exp(...) with fast exp and log;
                            1: theta - theta_ref from expm1 / log1p forms accurate
                            relative to the deviation, for slow diffusive flows
                            where neighbouring temperatures differ by ~1e-6 of
                            theta (FP32 thermal Couette 2 x 100: error 3e-3 ->
                            2e-4 of the temperature rise, ~1 % slower step) */
  int32_t feq_order;    /* 0 or 4: equilibrium and off-equilibrium populations
                           carry the fourth-order Hermite term xxyy (present
                           model, Sec. 2.3); 3: truncated at third order, as
                           in the original model the paper compares against
                           (Sec. 2.3, Table 1); with e1_centred = e2_off = 1
                           this is that model */
  int32_t steps_per_launch; /* 0: automatic (2 for FP32 domains periodic along both
                           axes with at least 900,000 nodes, else 1; batch
                           domains: 2 for every size, see hlbm_batch_step);
                           1: one step per kernel launch; 2: two
                           steps per launch, reading the state once and writing
                           it once every two steps (periodic along both axes
                           only, HLBM_EINVAL otherwise).  The per-node
                           arithmetic is the same either way (FP64 results
                           agree bitwise); hlbm_step runs an odd last step
                           alone.  tile_w / tile_h then apply to the two-step
                           sweep (tile_w 64 or 128 in FP64) */
} hlbm_params;

typedef struct hlbm_handle hlbm_handle;

/* Bytes of device workspace a domain with these parameters needs (two state
 * buffers of ten planes plus reduction scratch), or 0 if the parameters are
 * invalid.  Host-only; callable without a GPU. */
size_t hlbm_workspace_bytes(const hlbm_params *p);

/* Bytes of one raw state copy (ten planes, storage format) for
 * hlbm_save_state / hlbm_load_state; 0 if invalid.  Host-only.  State rows
 * are padded to a multiple of 64 elements and planes of 4 MiB or more to a
 * stride 64 KiB + 256 B past a multiple of 128 KiB, so this is
 * 10 x (pitch ny + padding) element sizes with pitch = nx rounded up to 64;
 * a copy is only meaningful to a domain with the same nx, ny and dtype. */
size_t hlbm_state_bytes(const hlbm_params *p);

/* Check parameters without touching the GPU: HLBM_OK or HLBM_EINVAL. */
int hlbm_validate(const hlbm_params *p);

/* Tile shape of hlbm_step's launches for these parameters (of the two-step
 * sweep when hlbm_launch_plan reports two steps per launch): tile_w / tile_h
 * as given, or the defaults when they are 0.  One step per launch:
 * 192-column tiles from 1024 columns, 128 below, 64 for nx <= 64; 16-row
 * strips at 192 columns in FP32, 32 otherwise, halved down to 4 rows until
 * about 768 workgroups exist in FP32 or 512 in FP64; never more rows than
 * ny.  Writes *host_tile_w and *host_tile_h; HLBM_OK, or HLBM_EINVAL if the
 * parameters are invalid or a pointer is NULL.  Host-only; callable without
 * a GPU. */
int hlbm_launch_shape(const hlbm_params *p, int32_t *host_tile_w, int32_t *host_tile_h);

/* Launch plan of hlbm_step for these parameters: steps per kernel launch (1
 * or 2, see steps_per_launch) and the tile shape of that launch (for two
 * steps per launch: tile_w / tile_h as given, or 184-column tiles from 1024
 * columns in FP32, with the tallest strips of 64, 32, 16 or 8 rows that give
 * at least 768 workgroups and fill the last round of 1024 resident ones at
 * least three quarters; 120 columns from 640 columns in FP32, halved down to
 * 8 rows until 768 workgroups exist; 128 columns otherwise, 64 for nx <= 64,
 * with 64-row strips halved down to 8 rows until about 384 workgroups
 * exist).  HLBM_OK, or
 * HLBM_EINVAL if the parameters are invalid or a pointer is NULL.
 * Host-only. */
int hlbm_launch_plan(const hlbm_params *p, int32_t *host_steps_per_launch, int32_t *host_tile_w,
                     int32_t *host_tile_h);

/* Initialise a domain from macroscopic fields (algorithm of Sec. 3.5, steps
 * 1-4): F0 = f^eq + f^1[a1FD] - psi/2 at every node, so the first step sees
 * the finite-difference off-equilibrium stress for any sigma.
 *   out        receives a new host handle (set to NULL on error)
 *   workspace  device buffer of at least hlbm_workspace_bytes(p) bytes, owned
 *              by the caller, that must outlive the handle
 *   rho, ux, uy, s  device [ny][nx] arrays (dtype of p): density, velocity,
 *              entropy s = c_v ln(theta / rho^(gamma-1))
 * Synchronises `stream` once to evaluate the initial CFL number.  Returns
 * HLBM_OK, HLBM_WARN_CFL (initialised; max local CFL >= 1), or an error. */
int hlbm_init(hlbm_handle **out, const hlbm_params *p, void *workspace, size_t ws_bytes,
              const void *rho, const void *ux, const void *uy, const void *s,
              hlbm_stream_t stream);

/* Enqueue nsteps (>= 0) time steps (Sec. 3.5, steps 5-11), one or two per
 * kernel launch as hlbm_launch_plan reports.  Asynchronous.
 * With bc_y = HLBM_BC_WALL every step (and hlbm_init) ends by rebuilding the
 * two wall rows, a regularised wet-node wall (our reading of the wall
 * condition of the thermal Couette case, Sec. 4.4, which the paper cites
 * without stating): rho_w from the populations with c_y = 0 plus twice those
 * that arrived from the interior; F = f^eq(rho_w, (wall_ux, 0), wall_theta) +
 * f^1[a1FD] with the velocity gradient zero along the wall and one-sided
 * second order across it, (-3 u_w + 4 u_1 - u_2) / 2; s from rho_w and
 * wall_theta.  The collision at wall nodes uses sigma = 1. */
int hlbm_step(hlbm_handle *h, int32_t nsteps, hlbm_stream_t stream);

/* Write the macroscopic fields of the current state: rho = sum F,
 * rho u = sum c F (Eqs. rhoalgo, ualgo), s, and theta from s and rho.
 * Any output pointer may be NULL.  Asynchronous. */
int hlbm_moments(hlbm_handle *h, void *rho, void *ux, void *uy, void *s, void *theta,
                 hlbm_stream_t stream);

/* Absolute populations F_i, device [9][ny][nx] in the handle's dtype
 * (HLBM_F32 storage deviations are added back to the reference).  Async. */
int hlbm_populations(hlbm_handle *h, void *F9, hlbm_stream_t stream);

/* Replace the state by absolute populations F9 [9][ny][nx] and entropy s
 * [ny][nx] (device, handle dtype).  Asynchronous. */
int hlbm_set_populations(hlbm_handle *h, const void *F9, const void *s, hlbm_stream_t stream);

/* Conservation totals in FP64, accumulated in a fixed order (deterministic):
 * host_out4 = {sum rho, sum rho u_x, sum rho u_y, sum(rho c_v theta +
 * rho |u|^2 / 2)}.  Synchronises `stream`. */
int hlbm_totals(hlbm_handle *h, double *host_out4, hlbm_stream_t stream);

/* Divergence check over the current state: HLBM_OK, or HLBM_EDIVERGED if any
 * node holds a non-finite value, rho <= 0 or theta <= 0.  If host_max_cfl is
 * not NULL it receives the largest local CFL number.  Synchronises `stream`. */
int hlbm_status(hlbm_handle *h, double *host_max_cfl, hlbm_stream_t stream);

/* Raw state copy for checkpoint / resume (bit-exact).  dst / src are device
 * buffers of hlbm_state_bytes(p) bytes.  Asynchronous. */
int hlbm_save_state(hlbm_handle *h, void *dst, hlbm_stream_t stream);
int hlbm_load_state(hlbm_handle *h, const void *src, hlbm_stream_t stream);

/* Number of steps taken since init (host counter). */
int64_t hlbm_steps_done(const hlbm_handle *h);

/* Release the host handle (the workspace stays the caller's). */
void hlbm_destroy(hlbm_handle *h);

/* Static message for a status code. */
const char *hlbm_strerror(int code);

/* For callers that cannot allocate device memory (no workspace, no handle,
 * e.g. under graph capture or in loops that must not call hipMalloc): the
 * conservation totals of hlbm_totals, computed from a raw state buffer
 * instead of a handle.  p: the domain's parameters (validated as by
 * hlbm_validate); state: device buffer of hlbm_state_bytes(p) bytes in the
 * storage format of hlbm_save_state (read only); host_out4 as in
 * hlbm_totals, with the same fixed-order FP64 reduction, so the same state
 * gives the same bits.  The reduction partials (1024 x 6 doubles, 48 KiB)
 * live in a fixed array of the library's own device memory, one per GPU,
 * held until the process ends; the call allocates nothing.  Every call on
 * one GPU shares that array: calls that overlap in time on one GPU (other
 * streams or host threads) race and must be serialised by the caller.  No
 * size limit beyond hlbm_validate's (the partial count does not depend on
 * the grid).  Synchronises `stream`.  HLBM_OK, HLBM_EINVAL (invalid
 * parameters or NULL pointer) or HLBM_EHIP. */
int hlbm_state_totals(const hlbm_params *p, const void *state, double *host_out4,
                      hlbm_stream_t stream);

/* Entropy from temperature, s = c_v ln(theta / rho^(gamma-1)) with
 * c_v = c_s^2 / (gamma - 1) (Sec. 2.1, 2.4), over n device elements of
 * `dtype`.  Asynchronous. */
int hlbm_entropy_from_theta(int32_t dtype, double gamma, const void *rho, const void *theta,
                            void *s, int64_t n, hlbm_stream_t stream);


/* ------------------------------------------------------------------------
 * Batched domains: many independent domains (each with its own hlbm_params,
 * all of one dtype) advanced together.  One step is ONE launch of a
 * persistent kernel whose workgroups walk a list of (domain, tile) items,
 * largest domains first; with use_graph the launches are replayed from a
 * captured hipGraph.  Fields of all domains are concatenated: domain k's
 * [ny_k][nx_k] block starts at element sum_{j<k} nx_j ny_j.  Each domain has
 * its own divergence flag; a diverged domain is frozen (its tiles are
 * skipped) while the others continue.
 * ------------------------------------------------------------------------ */
typedef struct hlbm_batch hlbm_batch;

/* Kernels of the batched step.  Both compute the step of Sec. 3 node by node
 * exactly as hlbm_step's one-step kernel does (FP64 results are bitwise
 * equal); they differ in how the work is cut:
 *   HLBM_BATCH_STRIPS  row strips of tile_w columns and tile_h rows swept
 *                      through the stages (two steps per launch when every
 *                      domain's own plan has two);
 *   HLBM_BATCH_TILES   tile_w x tile_h tiles whose halo is loaded at once:
 *                      less recomputed halo, for domains too small to give
 *                      long strips.  One step per launch, two for 32 x 16
 *                      and 64 x 8 tiles when every domain's own plan has
 *                      two (the first step then runs on the tile grown by
 *                      two nodes on every side, which yields the second
 *                      step's halo). */
typedef enum { HLBM_BATCH_STRIPS = 0, HLBM_BATCH_TILES = 1 } hlbm_batch_kernel;

/* Workspace bytes for `count` domains, or 0 if any parameter set is invalid,
 * has walls (bc_y = HLBM_BC_WALL is not available in batches) or the dtypes
 * differ.  Host-only. */
size_t hlbm_batch_workspace_bytes(const hlbm_params *params, int32_t count);

/* Initialise every domain as hlbm_init does.  params: host array of `count`;
 * rho, ux, uy, s: concatenated device fields.  Synchronises `stream`. */
int hlbm_batch_init(hlbm_batch **out, const hlbm_params *params, int32_t count, void *workspace,
                    size_t ws_bytes, const void *rho, const void *ux, const void *uy,
                    const void *s, hlbm_stream_t stream);

/* Enqueue nsteps steps of all domains.  When every domain takes two steps
 * per launch (FP32, periodic along both axes, steps_per_launch 0 or 2; the
 * size rule of single domains does not apply) the batch kernel advances two
 * steps per launch, else one.  use_graph = 1
 * (stream must not be NULL) replays a captured graph of sixteen launches
 * while enough steps remain, then one of two launches, and runs the rest
 * eagerly (an odd last step with a one-step launch); each graph is captured
 * on first use and again after the state has moved to the other buffer or
 * the tile shape changed.  HLBM_EHIP if a capture or launch fails. */
int hlbm_batch_step(hlbm_batch *b, int32_t nsteps, int32_t use_graph, hlbm_stream_t stream);

/* Concatenated macroscopic fields of all domains (NULL outputs skipped). */
int hlbm_batch_moments(hlbm_batch *b, void *rho, void *ux, void *uy, void *s, void *theta,
                       hlbm_stream_t stream);

/* Per-domain divergence flags (host_flags may be NULL); returns the number of
 * diverged domains (>= 0) or an error.  Synchronises `stream`. */
int hlbm_batch_status(hlbm_batch *b, int32_t *host_flags, hlbm_stream_t stream);

/* Kernel and tile shape of the batched step.  HLBM_BATCH_STRIPS: tile_w in
 * {64, 128, 192, 256} (64, 120, 128, 184 or 192 for two steps per launch,
 * 64 or 128 then in FP64), tile_h >= 4.  HLBM_BATCH_TILES: (tile_w, tile_h) in
 * {(32, 8), (32, 16), (64, 8), (32, 32), (64, 16)}, the first three in FP64.
 * HLBM_EINVAL for any other shape.  Drops the captured graphs.  Synchronises
 * `stream`. */
int hlbm_batch_set_shape(hlbm_batch *b, int32_t kernel, int32_t tile_w, int32_t tile_h,
                         hlbm_stream_t stream);

/* hlbm_batch_set_shape(b, HLBM_BATCH_STRIPS, tile_w, tile_h, stream). */
int hlbm_batch_set_tile(hlbm_batch *b, int32_t tile_w, int32_t tile_h, hlbm_stream_t stream);

/* Time `steps` steps (after one untimed launch; rounded up to even when the
 * strip kernel takes two steps per launch) for every shape that
 * hlbm_batch_set_shape accepts among strips {64, 120, 128, 184, 192, 256} x {4, 8, 16,
 * 32, 64, 128} and all tile shapes, twice each, keep the fastest and report
 * its kernel and shape (outputs may be NULL).  scratch: a device buffer of hlbm_batch_state_bytes(b) bytes
 * owned by the caller; the state at entry is saved there and loaded again
 * (divergence flags cleared) before every trial, so all shapes time the same
 * work, and once more at the end: the domains, their flags and the step
 * count are left as they were (the graphs are dropped and re-captured on the
 * next hlbm_batch_step).  HLBM_EINVAL if scratch is NULL.  Synchronises
 * `stream`. */
int hlbm_batch_autotune(hlbm_batch *b, int32_t steps, void *scratch, int32_t *host_best_kernel,
                        int32_t *host_best_w, int32_t *host_best_h, hlbm_stream_t stream);

/* Raw state of all domains (for checkpoint, or around hlbm_batch_autotune);
 * load also clears the divergence flags. */
size_t hlbm_batch_state_bytes(const hlbm_batch *b);
int hlbm_batch_save_state(hlbm_batch *b, void *dst, hlbm_stream_t stream);
int hlbm_batch_load_state(hlbm_batch *b, const void *src, hlbm_stream_t stream);

/* Steps per launch of the current batch kernel (2 for strips when every
 * domain's own plan is two steps per launch, else 1), the kernel
 * (hlbm_batch_kernel) and its tile shape.  Host-only. */
int hlbm_batch_plan(const hlbm_batch *b, int32_t *host_steps_per_launch, int32_t *host_kernel,
                    int32_t *host_tile_w, int32_t *host_tile_h);

int64_t hlbm_batch_nodes(const hlbm_batch *b);       /* sum of nx ny */
int64_t hlbm_batch_steps_done(const hlbm_batch *b);
void hlbm_batch_destroy(hlbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* HLBM_H */
