/*
 * hp_unet.h -- C ABI of the learned initial guess: a small U-Net trained and
 * run on the GPU by the library's own kernels, and the feature packing that
 * ties it to one propagation step (hp.h).
 *
 * This part is not in the paper.  It only supplies starting points for the
 * shifted solves (Zbar - b_k I) x_k = w of Sec. 2 (eq. W_k_def); hp_step_guess
 * judges every starting point by its FP64 residual and keeps the zero start
 * when the guess is worse, and the solves still stop on the paper's test, so
 * the network cannot change what a step computes, only how many GMRES
 * iterations (Sec. 4.2) it takes.
 *
 * What the network predicts.  With the free-space preconditioner M_k (Sec.
 * 4.2.2) and P = Zbar - Zbar_fs the medium part of the operator, the solution
 * is x_k = M_k^{-1} u_k with u_k = (I + P M_k^{-1})^{-1} w = w - P x_k.  The net
 * predicts the local correction u_k - w = -P x_k from planes that hold w,
 * y_k = M_k^{-1} w (the free-space solution), the medium V and the pole; the
 * guess is x0_k = M_k^{-1}(w + sigma_k net_k).
 *
 * Network: `levels` resolution levels with base * 2^l channels at level l; per
 * level two 3x3 convolutions (zero padding) each followed by ReLU, 2x2 average
 * pooling between levels, nearest-neighbour 2x upsampling concatenated
 * [upsampled, skip] on the way up, then two 3x3 convolutions with ReLU, and a
 * 1x1 output convolution without activation.  float32 weights and activations
 * with float32 accumulation; loss = mean squared error; Adam (Kingma & Ba 2015).
 *
 * Parameter layout (one flat float32 vector, the same on the host side): the
 * convolutions in the order enc_a[0], enc_b[0], ..., enc_a[L-1], enc_b[L-1],
 * dec_a[0], dec_b[0], ..., dec_a[L-2], dec_b[L-2], out; each one as weights
 * [cout][cin][k][k] (k = 3, or 1 for out) followed by bias [cout].  enc_a[0]
 * has `cin` inputs, enc_a[l] base*2^(l-1), dec_a[l] base*2^(l+1) + base*2^l.
 *
 * Tensors: device float32 NCHW [B][C][H][W]; fields: device complex128
 * (re, im) [ncomp][ny][nx] as in hp.h, batches of fields [B][ncomp][ny][nx].
 * Calls are asynchronous on the net's stream unless stated.  Return codes are
 * those of hp.h (HP_OK, HP_EINVAL, HP_ENOMEM, HP_EHIP).
 */
#ifndef HP_UNET_H
#define HP_UNET_H

#include "hp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hp_unet_s* hp_unet;

/* levels 1..6, base 1..256 channels, cin and cout 1..64.  Weights He-normal
 * (std sqrt(2 / fan_in), the output layer times 0.1) from a seeded generator,
 * biases 0, Adam moments 0.  stream: hipStream_t (NULL = default).  The net
 * owns its parameters and activations (reallocated when (B, H, W) changes). */
int hp_unet_create(int levels, int base, int cin, int cout, unsigned long long seed, void* stream, hp_unet* out);
long hp_unet_num_params(hp_unet net);

/* Arithmetic of the 3x3 convolutions (forward, data gradient and weight
 * gradient): HP_UNET_F32 (default): float32 direct convolution on the vector
 * ALUs; HP_UNET_BF16: implicit GEMMs on the matrix cores
 * (v_mfma_f32_16x16x32_bf16) with operands rounded to bf16 as they are staged
 * and float32 accumulation (the weight gradient contracts over pixels in
 * fixed splits summed in a fixed order, so repeated calls give identical
 * results).  Parameters, the 1x1 output layer, bias gradients and Adam stay
 * float32 in both. */
enum { HP_UNET_F32 = 0, HP_UNET_BF16 = 1 };
int hp_unet_set_precision(hp_unet net, int precision);

/* Host copies (each pointer may be NULL; arrays of hp_unet_num_params floats).
 * Synchronous.  get: parameters, gradients of the last hp_unet_grad, Adam
 * moments and step count; set: parameters and the Adam state (NULL moments
 * are zeroed), for checkpoint and resume. */
int hp_unet_get_params(hp_unet net, float* params, float* grads, float* adam_m, float* adam_v, long* adam_step);
int hp_unet_set_params(hp_unet net, const float* params, const float* adam_m, const float* adam_v, long adam_step);

/* y = net(x): x [B][cin][H][W], y [B][cout][H][W]; H, W multiples of
 * 2^(levels-1). */
int hp_unet_forward(hp_unet net, const float* x, int B, int H, int W, float* y);

/* Forward, loss = mean((net(x) - target)^2) over all B*cout*H*W outputs, and
 * the gradient of the loss with respect to every parameter (kept in the net
 * for hp_unet_adam / hp_unet_get_params).  loss: host, may be NULL (when given
 * the call synchronises). */
int hp_unet_grad(hp_unet net, const float* x, const float* target, int B, int H, int W, double* loss);

/* One Adam step with the gradients of the last hp_unet_grad:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps),
 * in float32 with 1-b1, 1-b2 and the bias corrections rounded from double. */
int hp_unet_adam(hp_unet net, double lr, double beta1, double beta2, double eps);

/* Scales of one step's guess features, on the device: scal[0] = rms of w,
 * scal[1] = rms of V over the unknowns, scal[2 + b] = rms of y_b, each at
 * least 1e-300.  V = (n^2 - n0^2)/n0^2, zero in the edge layer (distance
 * <= edge_width), exactly as in the operator.  w: one field; y: B fields
 * (y_b = M_{k_b}^{-1} w, e.g. from hp_apply_preconditioner); n2: device
 * [ny][nx]; scal: device, B + 2 doubles.  1 <= B <= 64. */
int hp_guess_stats(hp_unet net, int ncomp, int nx, int ny, double n0, int edge_width, const void* w, const void* y,
                   const double* n2, int B, double* scal);

/* Network input [B][4 ncomp + 3][ny][nx]: per component Re, Im of w / scal[0];
 * per component Re, Im of y_b / scal[2+b]; V / scal[1]; pole_feat[2b],
 * pole_feat[2b+1] (host, 2B doubles: features of sample b's pole, e.g.
 * asinh of Re and Im b_k) as constant planes.  Row 0 and column 0 are 0.  The
 * net must have cin = 4 ncomp + 3.  Synchronises the stream before reusing
 * its pinned feature buffer. */
int hp_guess_pack(hp_unet net, int ncomp, int nx, int ny, double n0, int edge_width, const void* w, const void* y,
                  const double* n2, const double* scal, const double* pole_feat, int B, float* x_in);

/* t_b = w + sigma_b net_out_b with sigma_b = scal[2+b] scal[1]; net_out
 * [B][2 ncomp][ny][nx] holds Re, Im per component; t: B fields.  The guess is
 * then x0_b = M_{k_b}^{-1} t_b (hp_apply_preconditioner). */
int hp_guess_unpack(hp_unet net, int ncomp, int nx, int ny, const void* w, const float* net_out, const double* scal,
                    int B, void* t);

/* Training target [B][2 ncomp][ny][nx] = -(P x_b) / sigma_b from px = P x_b
 * (B fields, hp_apply_medium of the solutions). */
int hp_guess_target(hp_unet net, int ncomp, int nx, int ny, const void* px, const double* scal, int B,
                    float* target);

/* Attach a trained net to a plan for HP_GUESS_LEARNED (hp_set_guess, hp.h):
 * the plan then computes every pole's starting point at the start of each step
 * itself (preconditioner solves, hp_guess_stats / pack, hp_unet_forward on
 * `chunk` poles at a time, hp_guess_unpack, preconditioner solves), on the
 * plan's stream, which must be the net's.  The net needs cin = 4 ncomp + 3,
 * cout = 2 ncomp, and nx, ny multiples of 2^(levels-1).  Allocates the guess
 * buffers (2 npoles + chunk complex128 fields and the network's input and
 * output for chunk poles; the net's activations are allocated by its first
 * forward pass at that shape), freed by hp_set_guess_net(plan, NULL, 0) or
 * with the plan.  The plan does not own the net: keep it alive while
 * attached.  chunk 1..64 (capped at npoles). */
int hp_set_guess_net(hp_plan plan, hp_unet net, int chunk);

const char* hp_unet_last_error(hp_unet net);
void hp_unet_destroy(hp_unet net);

#ifdef __cplusplus
}
#endif

#endif /* HP_UNET_H */
