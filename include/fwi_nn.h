/*
 * fwi_nn.h - C ABI of the kernels of the learned gradient preconditioner:
 * a small encoder-decoder CNN that maps (grad_eps, grad_sigma, eps_r, sigma)
 * to a model update, trained on gradient/update pairs from plain L-BFGS FWI
 * runs and used inside the inversion with plain L-BFGS as fallback.
 *
 * The paper itself has no such network: it only mentions machine-learning
 * assisted regularisation as related work (Sec. 1).  The inversion it
 * serves is the dual-parameter FWI loop of Sec. 3.1 (misfit Eq. (6),
 * gradients Eqs. (12)-(13)).
 *
 * Conventions
 * -----------
 * - Activations are NHWC, [N][H][W][C] bfloat16 (2 bytes, round to nearest
 *   even), C a multiple of 32 for every convolution operand.
 * - Convolution weights are [Co][3][3][Ci] bfloat16 (tap (ky, kx) reads the
 *   input pixel (y + ky - 1, x + kx - 1)); biases and all gradients of
 *   weights and biases are float32.  Every convolution is 3x3, stride 1,
 *   zero padding 1.  Products are exact in float32 and summed in float32
 *   on the matrix cores.
 * - Pointers are HIP device pointers owned by the caller; bfloat16 operands
 *   of the convolutions must be 16-byte aligned.  The library allocates
 *   nothing and keeps no state; scratch memory is a caller workspace.
 * - Every call is asynchronous on `stream` (a hipStream_t, NULL = the null
 *   stream) and returns FWI_NN_OK, FWI_NN_EINVAL for a null pointer, a bad
 *   size or misalignment (checked before anything is launched), or
 *   FWI_NN_EHIP when a launch fails.
 */
#ifndef FWI_NN_H
#define FWI_NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWI_NN_OK 0
#define FWI_NN_EINVAL (-1)
#define FWI_NN_EHIP (-5)
#define FWI_NN_MSE_BLOCKS 512   /* length of the partials array of fwi_nn_mse */

/* y = act(conv3x3(x, w) + bias), act = ReLU if relu != 0 else identity.
 * x [N][H][W][Ci], y [N][H][W][Co] bf16 (must not alias x); w [Co][3][3][Ci]
 * bf16; bias [Co] float32 or NULL.  Ci, Co multiples of 32; N * H * W < 2^36;
 * H, W <= 32768.
 * The input gradient of a convolution is fwi_nn_conv3x3 applied to the
 * output gradient with the weights from fwi_nn_flip (Ci and Co swapped). */
int fwi_nn_conv3x3(const void *x, const void *w, const float *bias, void *y, int32_t N,
                   int32_t H, int32_t W, int32_t Ci, int32_t Co, int32_t relu, void *stream);

/* wf[ci][2-ky][2-kx][co] = w[co][ky][kx][ci]: w [Co][3][3][Ci] -> wf
 * [Ci][3][3][Co], the weights of the transposed convolution. */
int fwi_nn_flip(const void *w, void *wf, int32_t Ci, int32_t Co, void *stream);

/* fwi_nn_flip for several layers in one launch: layer l's weights
 * w + off[l] ([co[l]][3][3][ci[l]], in elements) go flipped to wf + off[l].
 * off, ci, co: host arrays, read during the call; 1 <= nlayers <= 32, off
 * ascending with the layers disjoint (off[l] + 9 ci[l] co[l] <= off[l+1]),
 * 9 ci co < 2^31.  Elements of wf between the layers are not written. */
int fwi_nn_flip_layers(const void *w, void *wf, int32_t nlayers, const int64_t *off,
                       const int32_t *ci, const int32_t *co, void *stream);

/* Weight and bias gradients of y = conv3x3(x, w) + b given dz = dL/dy:
 *   dw[co][ky][kx][ci] = sum over pixels p of dz[p][co] x[p + (ky-1, kx-1)][ci],
 *   db[co] = sum_p dz[p][co]   (float32 outputs, overwritten).
 * The pixel sum is split over nsplit partial sums reduced in a fixed order,
 * so results are deterministic.  x and dz 16-byte aligned, N * H * W < 2^36,
 * H, W <= 32768, 1 <= nsplit <= 65535.  ws: device scratch of at least
 * fwi_nn_wgrad_workspace(Ci, Co, nsplit) bytes, 4-byte aligned. */
size_t fwi_nn_wgrad_workspace(int32_t Ci, int32_t Co, int32_t nsplit);
int fwi_nn_wgrad(const void *x, const void *dz, float *dw, float *db, int32_t N, int32_t H,
                 int32_t W, int32_t Ci, int32_t Co, int32_t nsplit, void *ws, size_t ws_bytes,
                 void *stream);

/* dz[i] = y[i] > 0 ? dy[i] : 0 over n bf16 values (y = the ReLU output). */
int fwi_nn_relu_bwd(const void *y, const void *dy, void *dz, size_t n, void *stream);

/* 2x2 average pooling x [N][H][W][C] -> y [N][H/2][W/2][C] (H, W even),
 * and its adjoint dy [N][H/2][W/2][C] -> dx [N][H][W][C] (dx = dy / 4 on
 * each of the four pixels). */
int fwi_nn_pool2(const void *x, void *y, int32_t N, int32_t H, int32_t W, int32_t C, void *stream);
int fwi_nn_pool2_bwd(const void *dy, void *dx, int32_t N, int32_t H, int32_t W, int32_t C,
                     void *stream);
/* The adjoint of the pooling plus a skip gradient: dx = pool2_bwd(dy) + skip,
 * skip [N][H][W][C] (NULL = none), rounded to bf16 once, the same values as
 * fwi_nn_pool2_bwd followed by fwi_nn_add. */
int fwi_nn_pool2_bwd_add(const void *dy, const void *skip, void *dx, int32_t N, int32_t H,
                         int32_t W, int32_t C, void *stream);

/* y [N][Ho][Wo][C] = nearest 2x upsampling of x [N][Ho/2][Wo/2][C] plus
 * skip [N][Ho][Wo][C] (NULL = no skip); fwi_nn_up2_bwd is the adjoint of
 * the upsampling: dx [N][Hi][Wi][C] = sum of each 2x2 block of dy
 * [N][2Hi][2Wi][C]. */
int fwi_nn_up2_add(const void *x, const void *skip, void *y, int32_t N, int32_t Ho, int32_t Wo,
                   int32_t C, void *stream);
int fwi_nn_up2_bwd(const void *dy, void *dx, int32_t N, int32_t Hi, int32_t Wi, int32_t C,
                   void *stream);

/* y[i] = a[i] + b[i] over n bf16 values (y may alias a or b). */
int fwi_nn_add(const void *a, const void *b, void *y, size_t n, void *stream);

/* Mean squared error of the first cout channels of y [P][C] (bf16) against
 * target [P][cout] (float32):
 *   *loss = 1/(P cout) sum (y - target)^2   (double, device),
 * and, if dy is not NULL, dy [P][C] = 2 (y - target) / (P cout) in those
 * channels and 0 in the others (bf16).  partials: device double scratch of
 * FWI_NN_MSE_BLOCKS entries. */
int fwi_nn_mse(const void *y, const float *target, void *dy, double *loss, double *partials,
               size_t P, int32_t C, int32_t cout, void *stream);

/* One Adam step (Kingma and Ba, bias-corrected) on n float32 parameters w
 * with gradient g and moments m, v (updated in place); step = 1, 2, ...
 * If wb is not NULL it receives the updated parameters rounded to bf16. */
int fwi_nn_adam(float *w, const float *g, float *m, float *v, void *wb, size_t n, float lr,
                float beta1, float beta2, float eps, int32_t step, void *stream);

/* b[i] = bf16(a[i]) over n values. */
int fwi_nn_to_bf16(const float *a, void *b, size_t n, void *stream);

/* Network input from float32 planes: planes [N][4][H][W] -> x [N][H][W][C]
 * bf16 with x[n][y][x][c] = planes[n][c][y][x] * scale[n * 4 + c] for
 * c < 4 and 0 for 4 <= c < C (C >= 4).  scale: device float [N][4]. */
int fwi_nn_pack4(const float *planes, const float *scale, void *x, int32_t N, int32_t H,
                 int32_t W, int32_t C, void *stream);

/* Network output to float32 planes: out [N][2][H][W] = y[n][y][x][c] *
 * scale[n * 2 + c] for c < 2 (y [N][H][W][C] bf16, C >= 2; scale: device
 * float [N][2]). */
int fwi_nn_unpack2(const void *y, const float *scale, float *out, int32_t N, int32_t H,
                   int32_t W, int32_t C, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FWI_NN_H */
