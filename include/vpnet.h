/*
 * vpnet.h - C ABI of the learned warm start in libvp: a 4-level convolutional
 * U-Net (channels 16/32/64/128, two 3x3 convolutions per level, 2x2 stride-2
 * down-sampling, 2x2 stride-2 transposed-convolution up-sampling, skip
 * concatenation, 1x1 output head) that maps 8 input channels (thickness,
 * concentration, wind, ocean current, previous velocity) to 5 output channels
 * (velocity and the dual stress pi of Sec. 4.2, eq. pi).  The network only
 * proposes the starting point of the Newton iteration of vp.h; Newton finishes
 * the solve and decides its accuracy.
 *
 * Arithmetic: BF16 activations and weights on the matrix cores (MFMA), FP32
 * accumulation; FP32 master weights, output head, loss and Adam.
 * Layouts: NHWC, input [B][H][W][8] FP32, output/target [B][H][W][5] FP32, all
 * device pointers on the stream given to vpnet_create.  H and W multiples of 8.
 * Return codes as in vp.h (0 OK, < 0 error; vpnet_last_error for text).
 */
#ifndef VPNET_H
#define VPNET_H

#include <stdint.h>

#include "vp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vpnet_s* vpnet;

/* Network for a fixed batch and spatial size.  VP_EINVAL if batch < 1 or H, W not
 * positive multiples of 8. */
int vpnet_create(int batch, int height, int width, void* hip_stream, vpnet* out);
void vpnet_destroy(vpnet net);
const char* vpnet_last_error(vpnet net);
/* Number of parameters (flat FP32 vector: per layer weights then bias). */
int64_t vpnet_param_count(vpnet net);
/* Copy parameters in/out (device FP32, vpnet_param_count entries); set resets Adam. */
int vpnet_set_params(vpnet net, const float* src);
int vpnet_get_params(vpnet net, float* dst);
/* Gradient of the last vpnet_backward (device FP32, flat like the parameters). */
int vpnet_get_grads(vpnet net, float* dst);
/* output = net(input). */
int vpnet_forward(vpnet net, const float* input, float* output);
/* Forward, mean-squared-error loss against target, backward (gradients kept in the
 * net).  loss (host, nullable) receives the loss; synchronises when requested. */
int vpnet_backward(vpnet net, const float* input, const float* target, float* loss);
/* One Adam step (beta 0.9/0.999, eps 1e-8) with learning rate lr on the last gradients. */
int vpnet_adam(vpnet net, float lr);
/* vpnet_backward followed by vpnet_adam. */
int vpnet_train_step(vpnet net, const float* input, const float* target, float lr, float* loss);

/* Solver <-> network glue (device arrays in the layouts of vp.h):
 * features: the 8 normalised input channels on the (nx/f) x (ny/f) grid of f x f
 *   cell blocks (node fields averaged to cells first): H/2, (A-0.85)/0.15,
 *   v_air/25, v_ocean/0.1, v_prev/0.3.  f must divide nx and ny.
 * targets:  training targets on the cell grid: cell mean of (v - v_prev) / 0.3 (the
 *   velocity change over the step; v_prev nullable = 0) and the mean of pi over the
 *   cell's 4 Gauss points.
 * guess:    v0 = v_prev + 0.3 * (sampled change) at the nodes (0 on the boundary;
 *   v_prev nullable = 0) and pi0 at the Gauss points (nullable), by bilinear
 *   sampling of a (wc x hc) cell-centred network output. */
int vpnet_features(int nx, int ny, int f, const double* H, const double* A, const double* v_air,
                   const double* v_ocean, const double* v_prev, float* out, void* hip_stream);
int vpnet_targets(int nx, int ny, const double* v, const double* pi, const double* v_prev, float* out,
                  void* hip_stream);
int vpnet_guess(int nx, int ny, const float* net_out, int wc, int hc, const double* v_prev, double* v0,
                double* pi0, void* hip_stream);

/* The learned start of the Newton solve (Sec. 4.2) for the step data of the last
 * vp_set_state on ctx: its features box-averaged onto the network's grid
 * (f = nx / width = ny / height cells per grid cell, an integer), one forward pass,
 * and the output sampled back onto the mesh as (v0, pi0) like vpnet_guess (v0 =
 * v_prev + change).  Then, of the starts in `candidates` (VPNET_START_* flags), the
 * one with the lowest energy Phi (eq. energy, the merit function of the Newton
 * line search) is written to v0 [(ny+1)(nx+1)][2] and pi0 [4][3][ny][nx] (device):
 * the learned start; the previous-step velocity v_prev with pi = tau/Delta (eq. pi);
 * or zero.  Ties go to the earlier of learned, previous, zero.  chosen (host,
 * nullable) receives the chosen flag.  Newton always finishes the solve.
 * Needs a batch-1 network, a Q1 context and one stream for both.  On a mesh finer
 * than the network's grid (f > 1: pooled inputs) the proposed change is damped,
 * v0 = v_prev + VPNET_POOLED_SCALE (proposal - v_prev), and pi0 is taken
 * consistent with v0 (pi = tau/Delta, eq. pi): box-averaged, the proposal misses
 * the fine-scale deformation, and at full size it costs Newton iterations
 * (measured at 1024^2 and 2048^2 with a 256^2 network: 167 against 170 Newton
 * and 3465 against 2504 Krylov iterations from zero over five workloads; damped
 * by 0.3, 22-25% less time than from zero over six held-out ones).  On meshes
 * more than VPNET_MAX_POOL times the network's grid per side (not measured) the
 * learned start is not a candidate and the network is not run.  Synchronises.
 * VP_EINVAL for null pointers, an empty candidate set, mismatched sizes or the
 * learned start alone on too fine a mesh; VP_ESTATE before vp_set_state;
 * VP_ENONFINITE if an energy is not finite. */
enum { VPNET_START_LEARNED = 1, VPNET_START_PREVIOUS = 2, VPNET_START_ZERO = 4 };
enum { VPNET_MAX_POOL = 8 };
#define VPNET_POOLED_SCALE 0.3
int vpnet_infer(vpnet net, vp_ctx ctx, int candidates, double* v0, double* pi0, int* chosen);

/* Activations of the last forward pass and their gradients from the last
 * vpnet_backward, exposed for verification.  act 0 is the network input, act
 * k >= 1 the (post-ReLU) output of the k-th layer in execution order (20 layers
 * before the output head): [B][H_l][W_l][C] with H_l, W_l the layer's level size.
 * y (device FP32, nullable) receives the stored BF16 values, g (device FP32,
 * nullable) the gradient of the loss with respect to them; count (host, nullable)
 * the number of entries.  VP_EINVAL for act out of range, VP_ESTATE for g before
 * any vpnet_backward. */
int vpnet_inspect(vpnet net, int act, float* y, float* g, int64_t* count);

/* The network's matrix-core GEMM, exposed for verification: C[M][N] (FP32) =
 * op(A) op(B) with BF16 A ([M][K], or [K][M] if a_trans) and B ([K][N], or [N][K]
 * if b_trans). */
int vpnet_gemm(const void* A, const void* B, float* C, int M, int N, int K, int a_trans,
               int b_trans, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* VPNET_H */
