/*
 * fwi_tv.h - C ABI of the total-variation regularisation term of the
 * dual-parameter FWI (arXiv 2506.20513, Sec. 3.4, Algorithm 3 and the
 * isotropic TV definition TV(X) = sum sqrt((Dx X)^2 + (Dy X)^2) after it).
 *
 * Algorithm 3 as computed here (the paper names the steps, not the
 * equations).  For each field X (eps_r or sigma, [ny][nx] float32), with
 * s = max |X| and Xn = X / s, a split-Bregman iteration of the TV-denoising
 * problem  min_U mu/2 ||U - Xn||^2 + TV(U)  with circular forward
 * differences Dx, Dy:  start U = Xn, Z = B = 0, then `iters` times
 *   R  = mu Xn - lam (bwd_x(Zx - Bx) + bwd_y(Zy - By))   (circular backward
 *        differences: the adjoint D^T (Z - B)),
 *   U <- (R + lam (4 U + sum of the 4 neighbours of U)) / (mu + 8 lam),
 *   Z <- shrink(D U + B, 1 / lam)   (isotropic soft threshold),
 *   B <- B + D U - Z,
 * and finally, with the scale restored,
 *   grad += weight * (X - s U).
 * The neighbour average with the centre weighted 4/8 is the linearised
 * (proximal) ADMM step, which converges to the TV-denoised model for every
 * mu, lam > 0; the term added is the gradient of the Moreau envelope of TV.
 *
 * Memory: X and grad are device arrays [nfield][ny][nx] owned by the
 * caller; grad is read and updated in place.  ws is device scratch of at
 * least fwi_tv_workspace_bytes(nfield, ny, nx) bytes, 256-byte aligned.
 * mu, lam, weight are host arrays of nfield values (per-field settings).
 * The call is asynchronous on `stream` (hipStream_t, NULL = null stream).
 *
 * Returns 0 (FWI_OK), -1 (FWI_EINVAL: null pointer, nfield outside
 * 1..FWI_TV_MAX_FIELDS, ny or nx < 2, ny * nx >= 2^31, iters < 1, a
 * non-positive mu or lam), -4 (FWI_ENOMEM: workspace missing, misaligned or
 * too small) or -5 (FWI_EHIP: a launch failed).  Checks run before any
 * launch.  An all-zero field contributes nothing.
 */
#ifndef FWI_TV_H
#define FWI_TV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWI_TV_MAX_FIELDS 4

size_t fwi_tv_workspace_bytes(int32_t nfield, int32_t ny, int32_t nx);

int fwi_tv_gradient(const float *X, float *grad, int32_t nfield, int32_t ny, int32_t nx,
                    const float *mu, const float *lam, const float *weight, int32_t iters,
                    void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FWI_TV_H */
