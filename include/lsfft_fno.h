/*
 * lsfft_fno.h -- C ABI of the learned nonlocal surrogate: a neural operator
 * whose hidden layers have the form of Eq. 6.10 (Sec. 6),
 *     z <- A(W z + b + K z),
 * A the exact GELU, W z + b a pointwise (local) layer and K an integral
 * operator with a learned kernel, applied as a periodic convolution in
 * Fourier space truncated to the low modes (the Fourier-neural-operator
 * family named in Sec. 6).  The surrogate maps a body force with compact
 * support sampled on an n^3 grid (cin channels) to the translation-averaged
 * strain on the same grid (cout channels), the dataset of Eqs. 3.7 and 6.4
 * compressed as in Fig. 5, blocks 2-3.
 *
 * Architecture (the paper fixes none; these are this library's choices):
 *   lift      pointwise cin -> width
 *   layers x  { K: keep modes kx in [0,M), ky, kz in [-M,M) of the
 *               half-spectrum of the (z,y,x) grid (x the real-to-half axis),
 *               per mode a learned complex width x width matrix,
 *               Y[o] = sum_i X[i] R[mode][i][o]; inverse transform with
 *               1/n^3 (kx = 0 weight 1, kx > 0 weight 2 on the real part);
 *               z <- GELU(W z + b + K z) }
 *   project   pointwise width -> hidden, GELU, pointwise hidden -> cout
 *   loss      mean over the batch of ||y - t|| / ||t||
 *   optimiser Adam with bias correction (complex weights as real pairs)
 * Mode index m = (iz * 2M + iy) * M + kx, iy and iz in [0, 2M) standing for
 * the signed wavenumbers 0..M-1, -M..-1.
 *
 * Arithmetic: every matrix product (pointwise layers, per-mode complex
 * products, and their gradients) runs on bf16 MFMA with fp32 accumulation,
 * operands rounded to bf16 to nearest even; the truncated transforms, GELU,
 * loss and Adam run in fp32 (loss sums in fp64).  Parameters are kept as an
 * fp32 master copy inside the handle.
 *
 * Layouts (all device pointers, fp32, C order, x fastest):
 *   x   [batch][cin][n][n][n]     y, t  [batch][cout][n][n][n]
 *   packed parameters: in this order, each C-contiguous,
 *     lift_w [width][cin], lift_b [width],
 *     per layer l: w [width][width], b [width], r [modes][width][width][2]
 *       (re, im), modes = 4 M^3,
 *     proj1_w [hidden][width], proj1_b [hidden],
 *     proj2_w [cout][hidden], proj2_b [cout].
 *
 * Ownership: the handle owns its parameters, optimiser state and activation
 * workspace (sized for max_batch); callers own x, y, t and parameter/gradient
 * buffers they pass.  Calls enqueue on the handle's stream (the caller's
 * stream given at creation) and return once their results are complete.
 * A handle is not re-entrant.
 *
 * Errors: LSFFT_E_ARG for a null handle or pointer, batch outside
 * [1, max_batch], or an unsupported architecture (n not in {8, 16, 32};
 * modes < 1 or 2 modes > n; width != 32; hidden not a multiple of 32 or
 * > 256; cin or cout outside [1, 32]; layers outside [1, 8]);
 * LSFFT_E_ALLOC / LSFFT_E_DEVICE for HIP failures.
 */
#ifndef LSFFT_FNO_H
#define LSFFT_FNO_H

#include <stdint.h>

#include "lsfft.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n;        /* grid points per axis */
  int modes;    /* M */
  int width;    /* channels of the hidden layers (32) */
  int hidden;   /* channels of the projection's inner layer */
  int cin, cout;
  int layers;
} lsfft_fno_arch;

typedef struct lsfft_fno_s* lsfft_fno_t;

/* Number of fp32 scalars of the packed parameter vector (0 if the
 * architecture is unsupported). */
int64_t lsfft_fno_param_count(const lsfft_fno_arch* arch);

/* Create a surrogate for batches of up to max_batch samples; parameters
 * start at zero (set them with lsfft_fno_set_params). */
lsfft_status lsfft_fno_create(lsfft_fno_t* out, const lsfft_fno_arch* arch, int max_batch, void* hip_stream);

/* Copy packed parameters in (device, fp32) and reset the optimiser state. */
lsfft_status lsfft_fno_set_params(lsfft_fno_t h, const float* params);

/* Copy the packed fp32 master parameters out (device). */
lsfft_status lsfft_fno_get_params(lsfft_fno_t h, float* params);

/* Inference: y = surrogate(x) for batch samples. */
lsfft_status lsfft_fno_forward(lsfft_fno_t h, int batch, const float* x, float* y);

/* Forward, loss (host, mean relative L2 error) and the gradient of the loss
 * with respect to every packed parameter; the gradient is kept in the handle
 * for lsfft_fno_adam and copied to `grad` (device, packed) when not NULL. */
lsfft_status lsfft_fno_loss_grad(lsfft_fno_t h, int batch, const float* x, const float* t, float* grad,
                                 double* loss);

/* One Adam step with the kept gradient (the step counter lives in the
 * handle and restarts with lsfft_fno_set_params). */
lsfft_status lsfft_fno_adam(lsfft_fno_t h, float lr, float beta1, float beta2, float eps);

/* lsfft_fno_loss_grad followed by lsfft_fno_adam. */
lsfft_status lsfft_fno_train_step(lsfft_fno_t h, int batch, const float* x, const float* t, float lr,
                                  double* loss);

lsfft_status lsfft_fno_destroy(lsfft_fno_t h);

#ifdef __cplusplus
}
#endif

#endif /* LSFFT_FNO_H */
