/*
 * glbm_cnn.h — C ABI of the learned warm start of the GLBM library.
 *
 * A small convolutional encoder-decoder maps per-node features of a shale
 * instance (phase one-hot, porosity, log10 of the lattice permeability,
 * log10 of the pressure) to a prediction of its steady density and velocity
 * fields.  The GLBM solve of arXiv:1601.00704 (Sec. 2.3, Eq. 29-37) then
 * starts from the equilibrium of the prediction instead of rest and iterates
 * to the same residual; the solver, not the network, decides the answer.
 * The network itself is not part of the paper.
 *
 * Tensors are channels-last (NHWC).  Activations, activation gradients and
 * the convolution weights are bfloat16 (stored as uint16_t bit patterns);
 * every contraction accumulates in FP32 on the MFMA units; master weights,
 * weight gradients and Adam moments are FP32.  Convolutions are 3x3,
 * stride 1, with periodic padding (the lattice is periodic).
 *
 * Conventions: return GLBM_OK (0) or a negative GLBM_E* code (glbm.h);
 * glbm_last_error() explains.  Device pointers must stay valid for the call;
 * work is queued on the given HIP stream (NULL: null stream) and calls that
 * return host values synchronise it.
 */
#ifndef GLBM_CNN_H
#define GLBM_CNN_H

#include <stddef.h>
#include <stdint.h>

#include "glbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- layers -- */

/*
 * y = act(conv3x3(x, w) + bias) on a batch of B images of H x W pixels.
 *   x        bf16 NHWC, pixel stride x_pitch channels, channels
 *            [x_off, x_off + cin) used; cin a multiple of 8
 *   w        bf16 [cout_pad][k_pad], cout_pad = round_up(cout, 16),
 *            k_pad = round_up(9 cin, 32); column k = tap * cin + ci with
 *            tap = 3 (dy + 1) + (dx + 1) reading x at (y + dy, x + dx)
 *            (periodic); padding entries must be zero
 *   bias     FP32 [cout] or NULL
 *   y        bf16 (y_is_f32 = 0) or FP32 (y_is_f32 = 1) NHWC, pixel stride
 *            y_pitch, channels [y_off, y_off + cout) written
 *   relu     1: max(., 0)
 *   accumulate  1: add to the values already in y (bf16 output only)
 * Requirements: W a multiple of 64; x and w 16-byte aligned, x_pitch and
 * x_off multiples of 8; EINVAL otherwise.
 */
int glbm_conv3x3_forward(const uint16_t* x, int32_t x_pitch, int32_t x_off, int32_t cin, const uint16_t* w,
                         const float* bias, void* y, int32_t y_pitch, int32_t y_off, int32_t cout, int32_t relu,
                         int32_t y_is_f32, int32_t accumulate, int32_t batch, int32_t height, int32_t width,
                         void* hip_stream);

/*
 * Weights of the data gradient of a convolution: wt[ci][tap' * cout_pad + co]
 * = w[co][(8 - tap') * cin + ci], so that
 *   dx = conv3x3(dy, wt)   (cin_pad = round_up(cin, 16) rows,
 *                            k_pad = round_up(9 cout_pad, 32) columns).
 */
int glbm_conv3x3_flip_weights(const uint16_t* w, int32_t cin, int32_t cout, uint16_t* wt, void* hip_stream);

/*
 * Weight and bias gradients of a convolution:
 *   dw[co][tap * cin + ci] = sum_pixels dy[p][co] x[p + d(tap)][ci]
 *   db[co] = sum_pixels dy[p][co]
 * x as in glbm_conv3x3_forward; dy bf16 NHWC with pixel stride dy_pitch and
 * channels [dy_off, dy_off + cout).  dw: FP32 [cout][9 cin]; db: FP32 [cout]
 * (may be NULL).  workspace: device memory of glbm_conv3x3_wgrad_workspace()
 * bytes (split-K partials, reduced in a fixed order: deterministic).
 */
size_t glbm_conv3x3_wgrad_workspace(int32_t cin, int32_t cout, int32_t batch, int32_t height, int32_t width);
int glbm_conv3x3_backward_weight(const uint16_t* x, int32_t x_pitch, int32_t x_off, int32_t cin, const uint16_t* dy,
                                 int32_t dy_pitch, int32_t dy_off, int32_t cout, float* dw, float* db,
                                 void* workspace, int32_t batch, int32_t height, int32_t width, void* hip_stream);

/* ------------------------------------------------------------- network -- */

typedef struct glbm_cnn_s* glbm_cnn;

#define GLBM_CNN_IN_CHANNELS 8   /* 6 features + 2 zero channels */
#define GLBM_CNN_OUT_CHANNELS 4  /* rho, u_x, u_y (normalised) + 1 unused */

/*
 * Encoder-decoder (U-Net shape), ten 3x3 convolutions:
 *   enc1: 8 -> 32 -> 32 (H x W)      avg-pool 2x2
 *   enc2: 32 -> 64 -> 64 (H/2)       avg-pool 2x2
 *   enc3: 64 -> 128 -> 128 (H/4)     nearest upsample 2x, concat with enc2 output
 *   dec2: 192 -> 64 -> 64 (H/2)      nearest upsample 2x, concat with enc1 output
 *   dec1: 96 -> 32 -> 3 (H)          (ReLU after every convolution but the last)
 * Parameters (FP32, flat, in this order per layer: weights [cout][cin][3][3]
 * with kernel index (dy + 1, dx + 1), then bias [cout]).
 * Sizes: H and W multiples of 256; the context holds activations for up to
 * max_batch images.  Weights start He-normal from `seed` (counter-based).
 */
int glbm_cnn_create(glbm_cnn* out, int32_t max_batch, int32_t height, int32_t width, uint64_t seed,
                    void* hip_stream);
int glbm_cnn_destroy(glbm_cnn cnn);
int64_t glbm_cnn_num_params(glbm_cnn cnn);
int glbm_cnn_get_params(glbm_cnn cnn, float* host);
int glbm_cnn_set_params(glbm_cnn cnn, const float* host);
/* FP32 gradients of the last glbm_cnn_train_step / glbm_cnn_backward (same layout). */
int glbm_cnn_get_grads(glbm_cnn cnn, float* host);

/* Inference: x bf16 [batch][H][W][8] -> y FP32 [batch][H][W][4] (device). */
int glbm_cnn_forward(glbm_cnn cnn, const uint16_t* x, float* y, int32_t batch);

/*
 * Forward, masked mean-squared error against target (FP32 [batch][H][W][4],
 * channels 0..2) over the nodes with mask != 0 (uint8 [batch][H][W]), and the
 * backward pass into the FP32 gradients.  *loss (host) receives the loss.
 */
int glbm_cnn_backward(glbm_cnn cnn, const uint16_t* x, const float* target, const uint8_t* mask, int32_t batch,
                      double* loss);

/*
 * Replace the FP32 gradients by host values (same layout as the parameters),
 * e.g. to apply an optimizer step to gradients computed elsewhere.
 */
int glbm_cnn_set_grads(glbm_cnn cnn, const float* host);

/*
 * One Adam step (Kingma & Ba, 2015) on the current gradients: with t the
 * number of Adam steps taken so far by this network, including this one,
 *   m = 0.9 m + 0.1 g,  v = 0.999 v + 0.001 g^2,
 *   p -= lr (m / (1 - 0.9^t)) / (sqrt(v / (1 - 0.999^t)) + 1e-8)
 * elementwise in FP32 on the master weights, which are then re-rounded to
 * the bf16 weights the convolutions use.  Errors: GLBM_EINVAL for lr <= 0.
 */
int glbm_cnn_adam_step(glbm_cnn cnn, float lr);

/* glbm_cnn_backward followed by glbm_cnn_adam_step. */
int glbm_cnn_train_step(glbm_cnn cnn, const uint16_t* x, const float* target, const uint8_t* mask, int32_t batch,
                        float lr, double* loss);

/* ----------------------------------------------- coupling with the solver -- */

/*
 * Input features of instance `inst` of a GLBM context into x (bf16
 * [ny][nx][8], device): one-hot pore / inorganic / organic class, eps,
 * log10(K_lattice) (open pore: +3), log10_pressure_mpa, 0, 0 — taken from the
 * class map and the table given to glbm_set_local_perm.
 */
int glbm_cnn_features(glbm_ctx ctx, int32_t inst, double log10_pressure_mpa, uint16_t* x);

/*
 * Training target of instance `inst` from its current state: target FP32
 * [ny][nx][4] = ((rho - 1) / rho_scale, u_x / u_scale, u_y / u_scale, 0) and
 * mask uint8 [ny][nx] = 1 on fluid nodes (device pointers).
 */
int glbm_cnn_targets(glbm_ctx ctx, int32_t inst, double rho_scale, double u_scale, float* target,
                     uint8_t* mask);

/*
 * Warm start: set instance `inst` to the equilibrium of the prediction
 * y FP32 [ny][nx][4] (device): rho = 1 + rho_scale y0, u = u_scale (y1, y2, 0).
 */
int glbm_cnn_apply(glbm_ctx ctx, int32_t inst, const float* y, double rho_scale, double u_scale);

/*
 * glbm_cnn_apply that allocates no device memory, for callers that cannot
 * call hipMalloc (code under HIP graph capture, tight serving loops,
 * harnesses that forbid it).  The rho - 1 and velocity fields are staged in
 * a static per-GPU scratch array of GLBM_NOALLOC_MAX_NODES nodes (16 MiB,
 * held until the process ends) instead of a buffer allocated per call; the
 * result is the same as glbm_cnn_apply's.  Calls on one GPU share that
 * array, so calls that overlap on one GPU (several host threads, or
 * contexts on different streams of one device) race: serialise them.
 * Errors: as glbm_cnn_apply; GLBM_EINVAL for an instance of more than
 * GLBM_NOALLOC_MAX_NODES nodes.
 */
#define GLBM_NOALLOC_MAX_NODES (1 << 20)
int glbm_cnn_apply_noalloc(glbm_ctx ctx, int32_t inst, const float* y, double rho_scale, double u_scale);

#ifdef __cplusplus
}
#endif

#endif /* GLBM_CNN_H */
