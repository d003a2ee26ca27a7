/*
 * epidmc_denoise.h -- C ABI of the learned denoiser of low-count EPID images.
 *
 * The paper proposes removing the statistical noise of a low-count Monte Carlo image with
 * a trained network, so that a short simulation plus one network pass stands in for a long
 * simulation (Sec. 4.1).  The paper gives no architecture; the one built here is a U-Net:
 *
 *   input      2 channels: image / s (s = the image's mean over the frame) and the
 *              radiological thickness (Sec. 2.2) / 20 cm; stored as 8 BF16 channels
 *              (6 zero) so that every channel count is a multiple of 8
 *   encoder    level l = 0..3, c_l = 32 * 2^l: conv3x3+ReLU, conv3x3+ReLU; 2x2 average
 *              pooling between levels
 *   decoder    level l = 2, 1, 0: conv1x1 (c_{l+1} -> c_l, no ReLU) of the level below,
 *              nearest 2x upsampling, concatenation [encoder level-l output, upsampled],
 *              conv3x3+ReLU (2 c_l -> c_l), conv3x3+ReLU
 *   head       conv1x1 (32 -> 1) added to the image channel; the result times s is the
 *              denoised image
 *   training   mean squared error against a high-count image (divided by the same s),
 *              Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights
 *
 * Arithmetic: BF16 weights and activations (round to nearest even), FP32 accumulation
 * (MFMA), FP32 biases, loss and gradient reductions, FP64 images at the boundary.
 *
 * Layout: activations are NHWC (image, row, column, channel) with a channel stride `ld`
 * (elements between consecutive pixels), so a tensor can be a channel slice of a wider
 * one; the kernels move 8 channels (16 bytes) at a time, so tensor pointers are 16-byte
 * aligned (a slice starts at a multiple of 8 channels).  Convolution weights are
 * [c_out][k][k][c_in].  BF16 values are passed as their
 * 16-bit patterns (uint16_t).  All pointers are device pointers unless stated; every
 * call is asynchronous on `stream` (a hipStream_t as void*, NULL = default stream) and
 * allocates no device memory: scratch buffers come from the caller.  Errors: epidmc_status
 * codes from epidmc.h; EPIDMC_E_ARG / E_SHAPE for invalid sizes, E_DEVICE for a launch
 * failure.
 */
#ifndef EPIDMC_DENOISE_H
#define EPIDMC_DENOISE_H
#include <stddef.h>
#include <stdint.h>

#include "epidmc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- layer operations ----------------------------------------------------------- */

/* y = act(conv_k(x, w) + bias), k = 1 or 3 ('same' zero padding), over n images of h x w
 * pixels.  c_in a multiple of 8, c_out a multiple of 32, ldx >= c_in, ldy >= c_out, both
 * multiples of 8.  bias may be NULL (no bias).  relu != 0 applies max(., 0).  gate, when
 * not NULL, zeroes every output element whose gate element (same pixel and channel,
 * stride ldg) is not > 0: the derivative of a ReLU, so that the call computes a
 * backward-data pass when w holds the flipped, transposed weights of epidmc_dn_weights. */
epidmc_status epidmc_dn_conv(const uint16_t *x, int ldx, int c_in, const uint16_t *w, const float *bias,
                             uint16_t *y, int ldy, int c_out, const uint16_t *gate, int ldg,
                             int n, int h, int w_px, int k, int relu, void *stream);

/* Weight gradient of conv_k: dw[o][i][j][c] = sum over pixels p of g[p][o] * x[p + (i, j)
 * - (k-1)/2][c] (FP32, [c_out][k][k][c_in]), and db[o] = sum_p g[p][o] (FP32; db may be
 * NULL).  c_in a multiple of 8, c_out a multiple of 32.  The sum is split over pixel
 * chunks whose FP32 partials go to `scratch` and are then added in a fixed order, so the
 * result is deterministic.  epidmc_dn_wgrad_scratch gives the floats `scratch` needs. */
epidmc_status epidmc_dn_wgrad_scratch(int n, int h, int w_px, int k, int c_in, int c_out, size_t *floats);
epidmc_status epidmc_dn_wgrad(const uint16_t *x, int ldx, int c_in, const uint16_t *g, int ldg, int c_out,
                              int n, int h, int w_px, int k, float *dw, float *db,
                              float *scratch, size_t scratch_floats, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): epidmc_dn_wgrad with the partial sums in
 * a scratch array that the library holds in device memory, one per GPU it runs on, until the
 * process ends; nothing is allocated or freed by the call.  Same arguments, kernels and
 * result as epidmc_dn_wgrad (bit for bit); returns EPIDMC_E_WORKSPACE when the shape needs
 * more than EPIDMC_DN_WGRAD_NOALLOC_FLOATS floats of scratch (epidmc_dn_wgrad_scratch gives
 * the need).  Every call on one GPU uses that GPU's array: calls that overlap on one GPU
 * (on different streams, or from different threads) race and must be serialised by the
 * caller.  The first call on a device resolves the array's address on the current device. */
#define EPIDMC_DN_WGRAD_NOALLOC_FLOATS (10u << 20) /* 40 MiB: every layer of the U-Net below for
                                                  * batches of up to 8 images of 1024 x 768 */
epidmc_status epidmc_dn_wgrad_noalloc(const uint16_t *x, int ldx, int c_in, const uint16_t *g, int ldg, int c_out,
                                      int n, int h, int w_px, int k, float *dw, float *db, void *stream);

/* BF16 copies of FP32 weights w [c_out][k][k][c_in]: w_fwd in the same layout, and w_bwd
 * [c_in][k][k][c_out] with the taps reversed (w_bwd[c][i][j][o] = w[o][k-1-i][k-1-j][c]),
 * the weights of the backward-data convolution.  Either output may be NULL. */
epidmc_status epidmc_dn_weights(const float *w, int c_out, int k, int c_in, uint16_t *w_fwd, uint16_t *w_bwd,
                                void *stream);

/* 2x2 average pooling of n images of h x w pixels (h, w even) and c channels (a multiple
 * of 8) into h/2 x w/2. */
epidmc_status epidmc_dn_pool(const uint16_t *x, int ldx, uint16_t *y, int ldy, int c, int n, int h, int w_px,
                             void *stream);
/* Nearest 2x upsampling of h x w pixels into 2h x 2w. */
epidmc_status epidmc_dn_upsample(const uint16_t *x, int ldx, uint16_t *y, int ldy, int c, int n, int h, int w_px,
                                 void *stream);
/* The adjoint of upsampling: y (h/2 x w/2) = sum of each 2x2 block of g (h x w, even). */
epidmc_status epidmc_dn_upsample_backward(const uint16_t *g, int ldg, uint16_t *y, int ldy, int c, int n, int h,
                                          int w_px, void *stream);
/* Gradient at an encoder output that feeds both a skip connection and the pooling: out =
 * (g_skip + g_pool(pixel / 2) / 4) where act > 0, else 0, over h x w pixels (even). */
epidmc_status epidmc_dn_skip_backward(const uint16_t *g_skip, int lds, const uint16_t *g_pool, int ldp,
                                      const uint16_t *act, int lda, uint16_t *out, int ldo, int c, int n, int h,
                                      int w_px, void *stream);

/* ---- the network ------------------------------------------------------------------ */
typedef struct epidmc_unet epidmc_unet;

epidmc_status epidmc_unet_create(epidmc_unet **out, int device);
epidmc_status epidmc_unet_destroy(epidmc_unet *u);
const char *epidmc_unet_last_error(const epidmc_unet *u);

/* Parameters are one flat FP32 vector: for each of the 18 layers in forward order
 * (e0a e0b e1a e1b e2a e2b e3a e3b u2 d2a d2b u1 d1a d1b u0 d0a d0b head): its weights
 * [c_out][k][k][c_in] at off_w and its biases at off_b.  The first layer's c_in is 8 (the
 * 2 input channels and 6 zero channels). */
epidmc_status epidmc_unet_param_count(const epidmc_unet *u, size_t *floats);
epidmc_status epidmc_unet_layer(const epidmc_unet *u, int layer, char name[8], int *k, int *c_in, int *c_out,
                                size_t *off_w, size_t *off_b);
int epidmc_unet_layers(const epidmc_unet *u);

/* Device memory for batches of up to n images of h x w pixels (h, w multiples of 8):
 * activations, gradients, weights and Adam moments.  Binding clears the parameters
 * (set them with epidmc_unet_set_params before use). */
epidmc_status epidmc_unet_workspace_size(const epidmc_unet *u, int n, int h, int w_px, size_t *bytes);
epidmc_status epidmc_unet_bind(epidmc_unet *u, void *dev_ptr, size_t bytes, int n, int h, int w_px, void *stream);

/* Load FP32 parameters (device pointer, param_count floats) and reset Adam's moments and
 * step count; read them back. */
epidmc_status epidmc_unet_set_params(epidmc_unet *u, const float *dev_params, void *stream);
epidmc_status epidmc_unet_get_params(const epidmc_unet *u, float *dev_params, void *stream);

/* Exponential moving average of the weights during training: with decay d in (0, 1), each
 * Adam step also sets ema <- d * ema + (1 - d) * theta; 0 (the default) turns it off.
 * set_params resets the average to the loaded parameters.  get_ema_params copies it out
 * (device pointer, param_count floats), e.g. to load it into an inference runner. */
epidmc_status epidmc_unet_set_ema(epidmc_unet *u, float decay);
epidmc_status epidmc_unet_get_ema_params(const epidmc_unet *u, float *dev_params, void *stream);

/* Denoise n <= bound images: noisy and thickness FP64 [n][h][w] (MeV per history and cm),
 * out FP64 [n][h][w] in the units of noisy. */
epidmc_status epidmc_unet_forward(epidmc_unet *u, const double *noisy, const double *thickness, double *out,
                                  int n, void *stream);
/* Loss (FP64 device scalar; may be NULL) and the gradient of the loss with respect to
 * every parameter (FP32, param_count floats, the parameter layout) for a batch of n
 * images with high-count targets FP64 [n][h][w]. */
epidmc_status epidmc_unet_gradient(epidmc_unet *u, const double *noisy, const double *thickness,
                                   const double *target, int n, float *dev_grad, double *loss, void *stream);
/* One Adam step of learning rate lr on a batch (the gradient as above, then the update). */
epidmc_status epidmc_unet_train_step(epidmc_unet *u, const double *noisy, const double *thickness,
                                     const double *target, int n, float lr, double *loss, void *stream);

#ifdef __cplusplus
}
#endif
#endif
