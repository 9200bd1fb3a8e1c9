/*
 * fadenoise: learned denoiser for low-sample renders of the light-stage face
 * renderer, on AMD Instinct MI355X.
 *
 * The paper names the sampling rate as the limitation of its method (Results
 * and Conclusion paragraph: more ray-traced samples cost more time).  This
 * library trades samples for a small convolutional encoder-decoder: a
 * 4-level U-Net (32, 64, 128, 256 channels; two 3x3 convolutions with leaky
 * ReLU per level; 2x2 average pooling down, nearest 2x upsampling and
 * channel concatenation of the skip up; a 1x1 output convolution) that maps
 * a low-spp render plus its albedo, normal and depth buffers to an estimate
 * of the converged image.  Radiance enters as log(1 + 16 x) (a fixed
 * exposure that brings the light stage's pixel values to order one), and
 * the output convolution predicts a correction of that input log-radiance.
 *
 * Convolutions run as implicit GEMMs on the matrix cores in bfloat16 with
 * fp32 accumulation (activations bfloat16, their gradients fp32 and rounded
 * to bfloat16 where they enter a product, weights kept in fp32 with bfloat16
 * copies); training uses Adam on a squared-error loss in log(1 + 16 x).
 *
 * Conventions: status 0 on success, negative on failure (FD_EINVAL -1,
 * FD_ENOMEM -2, FD_EDEVICE -3), message in fd_last_error; nothing throws.
 * Array arguments are DEVICE pointers (fp32, row-major [H][W][c]) read and
 * written on the stream set with fd_set_stream; calls return without
 * waiting.  The network owns its weights and scratch.  One network must not
 * be used from two host threads at once.
 */
#ifndef FADENOISE_H
#define FADENOISE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fd_net fd_net;

#define FD_IN_AUX 7   /* auxiliary channels: albedo rgb, normal xyz, depth */

/* Create a network for H x W images (H and W multiples of 8, at most 4096).
 * Weights start at zero; load them with fd_set_params.  Errors: FD_EINVAL,
 * FD_ENOMEM, FD_EDEVICE. */
int fd_create(int32_t height, int32_t width, fd_net **out);

/* The same for n images per call (n >= 1; for n > 1, H a multiple of 64;
 * n*H*W at most 22,369,621 pixels).  Every array argument of fd_forward,
 * fd_train_step and fd_backward_input then holds n images, [n][H][W][c],
 * and one call runs them all: each kernel launch covers every image, which
 * fills the chip where a single image's deep layers cannot.  Results per
 * image equal those of a one-image network; the training loss is the mean
 * over all n images' pixels.  fd_create(H, W) is fd_create_batch(H, W, 1).
 * Device memory grows with n (about 0.7 GB per 512 x 512 image). */
int fd_create_batch(int32_t height, int32_t width, int32_t n, fd_net **out);

/* Enqueue all later work on this HIP stream (hipStream_t). */
int fd_set_stream(fd_net *net, void *hip_stream);

/* Number of fp32 parameters (weights and biases of all layers). */
int64_t fd_num_params(const fd_net *net);

/* Parameter layout: for each layer in order (14 3x3 convolutions, then the
 * 1x1 output), weights [Cout][k*k][Cin] then bias [Cout]; the first layer's
 * Cin is 16 (10 used: log(1 + rgb), albedo, normal, depth; the rest zero).
 * fd_layer_shape gives layer i's (Cin, Cout, k) and returns 0, or FD_EINVAL
 * past the last layer. */
int fd_layer_shape(const fd_net *net, int32_t i, int32_t *cin, int32_t *cout, int32_t *k);

/* Copy all parameters in (params [fd_num_params], device) or out. Setting
 * them also resets the Adam moments and step count. */
int fd_set_params(fd_net *net, const float *params);
int fd_get_params(const fd_net *net, float *params);

/* Training state, for checkpoints: parameters, Adam moments m and v (each
 * [fd_num_params], device) and the step count.  fd_get_state copies them
 * out (any pointer may be NULL); fd_set_state restores them (params, m, v
 * all given).  Errors: FD_EINVAL (null net or, for fd_set_state, a null
 * array or step < 0). */
int fd_get_state(const fd_net *net, float *params, float *m, float *v, int32_t *step);
int fd_set_state(fd_net *net, const float *params, const float *m, const float *v, int32_t step);

/* Denoise: rgb [H][W][3] (the low-spp render), aux [H][W][7] (albedo,
 * normal, depth of the first hits, averaged over the pixel's samples) ->
 * out [H][W][3] radiance.  out may alias neither input. */
int fd_forward(fd_net *net, const float *rgb, const float *aux, float *out);

/* One training step on one image pair: forward, loss
 * mean over pixels and channels of (pred - log(1 + 16 target))^2 with pred the
 * network's log-radiance, backward, one Adam step (lr, betas 0.9 / 0.999,
 * eps 1e-8) on all parameters.  *loss_dev (device float, may be NULL) gets
 * the loss before the update.  grads (device, [fd_num_params], may be NULL)
 * gets the parameter gradient of this step. */
int fd_train_step(fd_net *net, const float *rgb, const float *aux, const float *target, float lr,
                  float *loss_dev, float *grads);

/* Gradient through the denoiser of the last fd_forward: dL_dout [H][W][3]
 * (the loss gradient with respect to that call's output radiance) ->
 * dL_drgb [H][W][3] (with respect to its rgb input, which must be passed
 * again, unchanged).  Parameters do not change.  This lets a fitting loop
 * take its data term on the denoised image and hand the renderer's adjoint
 * the gradient on the low-spp render.  Errors: -1 null argument, -4 no
 * prior fd_forward. */
int fd_backward_input(fd_net *net, const float *rgb, const float *dL_dout, float *dL_drgb);

/* Single layers: the kernels the network runs, callable on their own (for
 * element-wise checks of each kernel, or to compose other networks).  No
 * network is needed; work is enqueued on hip_stream (a hipStream_t, NULL for
 * the null stream).  Layouts as above: x [H][W][cin], y [H][W][cout],
 * weights [cout][9][cin] as bfloat16 bit patterns (the 16 high bits of the
 * fp32 value), tap t = 3 (dy + 1) + (dx + 1) reading pixel (y + dy, x + dx),
 * zero outside the image.
 *
 * fd_conv3x3: y = act(bias + conv(x, w)) in fp32 (before any rounding of
 * the stored activation), act = leaky ReLU (slope 0.01) when relu, else the
 * identity; bias may be NULL.  x is bfloat16 bit patterns, or fp32 (rounded
 * to bfloat16 as it is read) when x_is_f32 - the form the input-gradient
 * pass takes, with the flipped weights.  cin a multiple of 16.
 *
 * fd_conv3x3_wgrad: dw[co][t][ci] = sum_p g[p][co] x[nbr(p, t)][ci] (g fp32,
 * rounded to bfloat16 as it is read; x bfloat16), db[co] = sum_p g[p][co]
 * (db may be NULL).  Both are overwritten; sums are fp32 in an order that
 * varies between runs.  cin and cout multiples of 8.
 *
 * Errors: FD_EINVAL (sizes, null arrays), FD_EDEVICE. */
int fd_conv3x3(void *hip_stream, int32_t H, int32_t W, int32_t cin, int32_t cout, const void *x, int32_t x_is_f32,
               const uint16_t *w, const float *bias, int32_t relu, float *y);
int fd_conv3x3_wgrad(void *hip_stream, int32_t H, int32_t W, int32_t cin, int32_t cout, const uint16_t *x,
                     const float *g, float *dw, float *db);

const char *fd_last_error(const fd_net *net);
void fd_destroy(fd_net *net);

#ifdef __cplusplus
}
#endif
#endif
