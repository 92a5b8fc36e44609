/*
 * hlbm_nn.h -- C ABI of the learned closure of the hybrid-LBM library.
 *
 * The paper (arXiv 2002.03644) has no learned component; this part adds one
 * beside the method.  A coarse HLBM run is corrected after every step by a
 * small convolutional network that predicts, from the coarse moments
 * X = (rho, u_x, u_y, theta), the increment that brings them towards the
 * restriction of a fine-grid HLBM run of the same flow.  The fine run is both
 * the source of the training targets and the reference for the error.
 *
 * Network: three 3x3 convolutions 4 -> 32 -> 32 -> 4 with periodic padding
 * and ReLU after the first two (11 588 parameters), on per-channel
 * standardised inputs, predicting standardised increments:
 *   y = (CNN((X - in_mean) / in_std)) * out_std + out_mean.
 * Arithmetic: BF16 operands on the matrix cores with FP32 accumulation;
 * BF16 activations; FP32 master parameters, Adam moments, loss and gradients.
 * Training minimises the mean squared error over all standardised output
 * elements with Adam (Kingma and Ba, with bias correction).
 *
 * Conventions as in hlbm.h: device pointers unless named host_, caller-owned
 * workspace (the library never allocates device memory), asynchronous work
 * on `stream`, negative hlbm_status_code on error, no overlapping calls on one
 * handle from several host threads.
 *
 * Field batches: element (sample s, channel c, node i) of a batch of
 * [ny][nx] fields sits at ptr[s * s_stride + c * c_stride + i] (float), with
 * channels (rho, u_x, u_y, theta) for inputs and their increments for
 * outputs.  A batch entry b reads sample idx[b] when idx (a device int32
 * array of `batch` entries) is given, sample b otherwise.
 */
#ifndef HLBM_NN_H
#define HLBM_NN_H

#include "hlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define HLBM_CNN_PARAMS 11588  /* W1[3][3][4][32] b1[32] W2[3][3][32][32] b2[32]
                                  W3[3][3][32][4] b3[4], W[dy][dx][c_in][c_out] with
                                  out[y][x] = b + sum in[y+dy-1][x+dx-1] W[dy][dx] */

typedef struct hlbm_cnn hlbm_cnn;

/* Workspace bytes for batches of up to max_batch fields of ny x nx, or 0 if
 * the sizes are invalid: nx a multiple of 32, ny a multiple of 4, both
 * >= 4, max_batch >= 1, max_batch * nx * ny < 2^31.  Host-only. */
size_t hlbm_cnn_workspace_bytes(int32_t max_batch, int32_t ny, int32_t nx);

/* Create a network on a workspace (256-byte aligned, at least the size
 * above) with the canonical parameters `params` (device, HLBM_CNN_PARAMS
 * floats, copied), zero Adam state and identity standardisation. */
int hlbm_cnn_init(hlbm_cnn **out, int32_t max_batch, int32_t ny, int32_t nx, void *workspace,
                  size_t ws_bytes, const float *params, hlbm_stream_t stream);

/* Replace the parameters (device, canonical order) and reset Adam. */
int hlbm_cnn_set_params(hlbm_cnn *c, const float *params, hlbm_stream_t stream);

/* Copy the current parameters / the gradient of the last hlbm_cnn_loss_grad
 * (canonical order) to dst (device, HLBM_CNN_PARAMS floats). */
int hlbm_cnn_get_params(hlbm_cnn *c, float *dst, hlbm_stream_t stream);
int hlbm_cnn_get_grads(hlbm_cnn *c, float *dst, hlbm_stream_t stream);

/* Standardisation: host_norm = in_mean[4], in_std[4], out_mean[4],
 * out_std[4] (std > 0).  Host-side; applies to calls enqueued afterwards. */
int hlbm_cnn_set_norm(hlbm_cnn *c, const float *host_norm);

/* Bound on the standardised output of hlbm_cnn_forward (and so of the
 * closure's increments): each channel's CNN output is clamped to
 * [-clip, clip] before de-standardising; 0 (the default) disables it.
 * Training (hlbm_cnn_loss_grad) never clamps.  Host-side. */
int hlbm_cnn_set_output_clip(hlbm_cnn *c, float clip);

/* Inference kernel: enable = 1 (the default) runs the three layers in one
 * kernel with the activations in LDS whenever nx is a multiple of 64 and no
 * idx is given; enable = 0 always runs one kernel per layer through the
 * workspace.  Both give identical results.  Host-side. */
int hlbm_cnn_set_fused(hlbm_cnn *c, int32_t enable);

/* Inference: y = CNN(x) for `batch` (1..max_batch) fields, written to y in
 * raw units.  x and y must not overlap. */
int hlbm_cnn_forward(hlbm_cnn *c, const float *x, int64_t x_sstride, int64_t x_cstride,
                     const int32_t *idx, int32_t batch, float *y, int64_t y_sstride,
                     int64_t y_cstride, hlbm_stream_t stream);

/* Forward and backward pass on (x, target): target holds raw increments
 * (standardised inside with out_mean, out_std) and shares x's idx.  Leaves
 * the parameter gradient in the handle and, if loss is not NULL, writes the
 * mean squared error (float, device) there. */
int hlbm_cnn_loss_grad(hlbm_cnn *c, const float *x, int64_t x_sstride, int64_t x_cstride,
                       const float *target, int64_t t_sstride, int64_t t_cstride,
                       const int32_t *idx, int32_t batch, float *loss, hlbm_stream_t stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the stored
 * gradient; returns the new step count (>= 1) or an error. */
int hlbm_cnn_adam(hlbm_cnn *c, float lr, hlbm_stream_t stream);

/* hlbm_cnn_loss_grad followed by hlbm_cnn_adam. */
int hlbm_cnn_train_step(hlbm_cnn *c, const float *x, int64_t x_sstride, int64_t x_cstride,
                        const float *target, int64_t t_sstride, int64_t t_cstride,
                        const int32_t *idx, int32_t batch, float lr, float *loss,
                        hlbm_stream_t stream);

void hlbm_cnn_destroy(hlbm_cnn *c);

/* Restriction of fine fields to a grid coarser by `factor` (ny, nx
 * multiples of it): block means rho_c = <rho>, u_c = <rho u> / <rho>,
 * theta_c = <rho theta> / <rho> over factor x factor cells, which keep each
 * block's mass, momentum and pressure.  Inputs: `batch` fine fields
 * concatenated, [batch][ny][nx] each (as hlbm_batch_moments writes them);
 * output element (b, c, i) at out[b * o_sstride + c * o_cstride + i]. */
int hlbm_restrict(const float *rho, const float *ux, const float *uy, const float *theta,
                  int32_t batch, int32_t ny, int32_t nx, int32_t factor, float *out,
                  int64_t o_sstride, int64_t o_cstride, hlbm_stream_t stream);

/* Apply increments to every domain of an HLBM_F32 batch whose domains all
 * have one size n = nx ny.  x: the current moments (rho, u_x, u_y, theta),
 * delta: the increments, both [4][count][n] (channel stride count n, domain
 * stride n, as hlbm_batch_moments writes them with one plane per channel).
 * conserve = 1 shifts the density and momentum increments by their domain
 * means so total mass and momentum stay unchanged.  Only the equilibrium part
 * of the populations moves (F += f^eq(X') - f^eq(X)); the entropy follows
 * X'. */
int hlbm_batch_correct(hlbm_batch *b, const float *x, const float *delta, int32_t conserve,
                       hlbm_stream_t stream);

/* ncycles correction cycles of an HLBM_F32 batch: each is `every` (>= 1)
 * batch steps, then the moments, the network's increment and
 * hlbm_batch_correct.  The network must have been created for max_batch >=
 * count and the domains' ny x nx, and trained for increments over `every`
 * steps; its workspace holds the moments and increments.  use_graph = 1
 * replays captured hipGraphs of eight cycles while that many remain, then
 * of two, and runs the rest eagerly (stream must not be NULL).  With
 * the HLBM_BATCH_TILES kernel (hlbm_batch_set_shape) the same results come
 * with fewer passes over the state: a cycle's last step also writes the
 * moments, and a cycle's correction is applied by the next cycle's first
 * step as it loads the state (the last cycle's by a pass of its own before
 * the call returns); a frozen domain's moments are then not refreshed. */
int hlbm_closure_step(hlbm_batch *b, hlbm_cnn *c, int32_t ncycles, int32_t every,
                      int32_t conserve, int32_t use_graph, hlbm_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* HLBM_NN_H */
