/*
 * gkb_cnn.h -- the learned inner preconditioner of the GKB solver (gkb.h):
 * a small convolutional network C_theta trained on residual / error pairs
 * that the solver's own multigrid-preconditioned inner solves generate, and
 * used inside flexible CG as  z = V(r) + (s / lambda) C_theta(rt / s),
 * V = one multigrid V-cycle, rt = r - M V(r) the residual the V-cycle leaves,
 * s = RMS of rt, lambda = mean of diag(W).
 * Plain multigrid-PCG is the fallback when the network's direction fails a
 * descent, progress or energy-gain test (gkb_stats_t.learned_solves).  (The paper's inner solver is any Krylov method
 * with a swappable preconditioner, Section 3; the network itself has no
 * counterpart in the paper.)
 *
 * Network: L convolution layers, kernel 3x3 (2D) or 3x3x3 (3D), 'same' zero
 * padding, bias, ReLU between layers, at most 16 channels per layer.
 * Input channels: the components of rt on the faces below / left of each
 * cell (u, v[, w]) divided by s, then log(mu) of the cell; output channels:
 * the correction of the same faces.  Arithmetic: BF16 weights and
 * activations on MFMA (v_mfma_f32_16x16x16_bf16) with FP32 accumulation;
 * FP32 master weights and Adam state.
 *
 * Parameter layout (flat FP32, per layer l): W_l[tap][c_in][c_out] then
 * b_l[c_out]; tap = (dz+1)*9 + (dy+1)*3 + (dx+1) (3D), (dy+1)*3 + (dx+1)
 * (2D).  Activations: channels-last FP32 [batch][(nz,) ny, nx][c] in device
 * memory.
 *
 * All pointers are device pointers unless marked host.  Calls are
 * synchronous: the calls that read device buffers (forward, backward, train,
 * eval) first wait for all work already submitted to the device, so buffers
 * written on any stream are complete, and return when their own work is
 * done.  Errors as in gkb.h (GKB_EINVAL, GKB_ENOMEM, GKB_EHIP); a call (or
 * an attach) whose points (batch * nx * ny * nz) exceed 2^31 - 1 returns
 * GKB_EINVAL.
 */
#ifndef GKB_CNN_H
#define GKB_CNN_H

#include <stddef.h>

#include "gkb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gkb_cnn gkb_cnn;

/* channels: host array of n_layers+1 channel counts (1..16 each).  Weights
   are initialised with a seeded He-uniform draw (seed) and zero biases. */
int gkb_cnn_create(int dim, int n_layers, const int *channels, unsigned seed, gkb_cnn **out);
void gkb_cnn_destroy(gkb_cnn *n);
long gkb_cnn_param_count(const gkb_cnn *n);

/* copy the flat FP32 parameter vector from / to HOST memory */
int gkb_cnn_set_params(gkb_cnn *n, const float *host_params);
int gkb_cnn_get_params(const gkb_cnn *n, float *host_params);

/* y = C_theta(x) for a batch of `batch` grids of nx * ny * nz points (nz = 1
   in 2D); x [batch][points][c_0], y [batch][points][c_L], FP32. */
int gkb_cnn_forward(gkb_cnn *n, int nx, int ny, int nz, int batch, const float *x, float *y);

/* Gradient of sum(dy .* C_theta(x)) with respect to the parameters (grad,
   HOST, param_count floats) and to x (dx, device, may be NULL); recomputes
   the forward pass. */
int gkb_cnn_backward(gkb_cnn *n, int nx, int ny, int nz, int batch, const float *x,
                     const float *dy, float *dx, float *grad_host);

/* One Adam step (lr, beta1, beta2, eps) with the HOST gradient `grad_host`
   (NULL: the gradient of the last gkb_cnn_train_step). */
int gkb_cnn_adam_step(gkb_cnn *n, const float *grad_host, double lr, double beta1,
                      double beta2, double eps);

/* Training on stored pairs.  inputs [n_pairs][points][c_0] and targets
   [n_pairs][points][c_L] (FP32, normalised as the preconditioner uses them)
   on full grids of nx * ny * nz points.  Runs `steps` Adam steps on batches
   of `batch` random crops of side `crop` (pair and origin drawn from a
   seeded generator), loss = mean squared error over all batch entries
   (inputs and targets are already normalised by the residual scale).
   loss_host (may be NULL) receives the loss of every step. */
int gkb_cnn_train(gkb_cnn *n, const float *inputs, const float *targets, int n_pairs, int nx,
                  int ny, int nz, int crop, int batch, int steps, double lr, unsigned seed,
                  float *loss_host);

/* Mean loss of the network on all stored pairs (full grids). */
int gkb_cnn_eval(gkb_cnn *n, const float *inputs, const float *targets, int n_pairs, int nx,
                 int ny, int nz, double *loss);

/* Versioned binary checkpoint: header, architecture, FP32 parameters, Adam
   moments and step count. */
int gkb_cnn_save(const gkb_cnn *n, const char *path);
int gkb_cnn_load(const char *path, gkb_cnn **out);

/* Use network n (kept by reference; must outlive the context or be detached
   with n = NULL) in the context's GKB_INNER_LEARNED inner solves. */
int gkb_attach_cnn(gkb_ctx *c, gkb_cnn *n);

/* Pair capture: while enabled, every inner solve of gkb_solve runs
   un-captured MG-PCG, snapshots the residual r_i and iterate x_i at the
   iterations listed in iters (host, n_iters entries, 0 = the start), and
   after convergence (x*) stores for each snapshot
       input  = pack(rt_i) / s_i,  target = pack(x* - x_i - V(r_i)) * lambda / s_i
   with rt_i = r_i - M V(r_i), s_i = RMS(rt_i), into inputs / targets ([max_pairs][cells][c]
   layout of gkb_cnn_train, c_0 = dim + 1 input channels, dim targets).
   Capture stops when max_pairs are stored.  inputs = NULL disables it.
   *count (host) receives the number of pairs stored so far. */
int gkb_set_capture(gkb_ctx *c, float *inputs, float *targets, int max_pairs, int n_iters,
                    const int *iters);
int gkb_capture_count(const gkb_ctx *c, int *count);

#ifdef __cplusplus
}
#endif

#endif /* GKB_CNN_H */
