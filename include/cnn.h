/*
 * cnn.h -- C ABI of the warm-start network kernels in libmoc (gfx950).
 *
 * A small convolutional network predicts the scalar flux of a lattice from its
 * rasterised cross sections; the prediction is handed to moc_set_initial_guess and
 * the plain power iteration (moc_solve) still decides convergence. This is a
 * project addition; the paper itself accelerates with CMFD (Sec. 2.1.2, Alg. MOCHFEM_CMFD).
 *
 * Conventions:
 *   - Activations are NHWC: [N][H][W][C], C fastest. BF16 tensors are passed as
 *     uint16_t bit patterns (bfloat16: the upper half of an IEEE float).
 *   - Convolutions are 3x3, stride 1, zero padding ("same"); weights are
 *     W[co][tap][ci] with tap = 3 ky + kx, i.e. z[n,y,x,co] = b[co] +
 *     sum W[co][3 ky + kx][ci] x[n, y + ky - 1, x + kx - 1, ci].
 *   - Channel counts: Ci a multiple of 32, Co a multiple of 16 (pad with zeros).
 *   - All pointers are device pointers on the current HIP device unless stated;
 *     calls enqueue on `stream` (NULL = the null stream) and return without waiting.
 *   - Return MOC_OK (0) or MOC_EINVAL (bad sizes or null pointers) / MOC_EHIP.
 */
#ifndef CNN_H
#define CNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* y = act(conv3x3(x, w) + bias): BF16 operands, FP32 accumulation on the matrix cores
 * (implicit GEMM: M = pixels, N = Co, K = 9 Ci). Tap (ky, kx) reads pixel
 * (y + (ky - 1) d, x + (kx - 1) d) for dilation d >= 1, zero outside the image, so the
 * output has the input's size. bias may be NULL. relu != 0 applies max(0, .). Writes
 * y_bf16 [N][H][W][Co] and/or y_f32 (either may be NULL). MOC_EINVAL for bad sizes
 * (Ci % 32, Co % 16 and Co / 16 in {1, 2, 4}) or d < 1. */
int cnn_conv3x3_forward(const uint16_t *x, const uint16_t *w, const float *bias, int32_t N,
                        int32_t H, int32_t W, int32_t Ci, int32_t Co, int32_t dilation, int32_t relu,
                        uint16_t *y_bf16, float *y_f32, void *stream);

/* Weight layout for the input gradient: wt[ci][tap][co] = bf16(w[co][8 - tap][ci]) from
 * FP32 w [Co][9][Ci]; then dx = cnn_conv3x3_forward(dz, wt, NULL, ..., Ci'=Co, Co'=Ci,
 * same dilation). */
int cnn_weights_for_dgrad(const float *w, int32_t Co, int32_t Ci, uint16_t *wt, void *stream);

/* Weight gradient, accumulated: dw[co][tap][ci] += sum_{n,y,x} dz[n,y,x,co]
 * x[n, y + (ky-1) d, x + (kx-1) d, ci] (BF16 operands on the matrix cores, FP32
 * accumulation; dw FP32, caller zeroes it; dilation d >= 1). */
int cnn_conv3x3_wgrad(const uint16_t *x, const uint16_t *dz, int32_t N, int32_t H, int32_t W,
                      int32_t Ci, int32_t Co, int32_t dilation, float *dw, void *stream);

/* db[co] += sum over pixels of dz (FP32 dz [npix][Co]). */
int cnn_bias_grad(const float *dz, int64_t npix, int32_t Co, float *db, void *stream);

/* Through a ReLU: dz = dy * (y > 0), y the layer's BF16 output. Writes FP32 and BF16. */
int cnn_relu_backward(const float *dy, const uint16_t *y, int64_t n, float *dz_f32, uint16_t *dz_bf16,
                      void *stream);

/* Mean squared error over the first `cv` of every `cs` channels (the rest are padding):
 * dy = 2 (y - t) / count on those channels, 0 elsewhere; loss_partials[block] receives
 * per-block sums of squares (nblocks = 256; the caller sums and divides by count). */
int cnn_mse_grad(const float *y, const float *t, int64_t npix, int32_t cs, int32_t cv, float *dy,
                 double *loss_partials, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): cnn_mse_grad without the workspace. Same dy;
 * loss (device FP64, one value) receives the mean squared error, the partial sums
 * divided by npix * cv. The 256 per-block partials live in a fixed 2 KiB array inside
 * the library (one per device, kept until the process ends; its size does not depend on
 * the input, so every size cnn_mse_grad accepts is accepted). Nothing is allocated.
 * Calls that overlap on one device (other streams, other threads) share that array and
 * race; serialise them. MOC_EINVAL for bad sizes or null pointers, MOC_EHIP if the
 * array's device address cannot be obtained or the launch fails. */
int cnn_mse_grad_noalloc(const float *y, const float *t, int64_t npix, int32_t cs, int32_t cv, float *dy,
                         double *loss, void *stream);

/* Adam with bias correction (step t >= 1) on FP32 master parameters p; also writes the
 * BF16 copy p_bf16 (may be NULL). */
int cnn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float beta1,
             float beta2, float eps, int32_t t, uint16_t *p_bf16, void *stream);

/* BF16 copy of FP32 data. */
int cnn_to_bf16(const float *src, int64_t n, uint16_t *dst, void *stream);

/* Input features of the warm-start network per material (device pointers, FP64 inputs
 * sigma_t [M][G], sigma_s [M][G][G] (from g to g'), nu_sigma_f [M][G], chi [M][G];
 * output FP32 features [M][4 G]): the log of the material's normalised infinite-medium
 * spectrum phi, (diag(Sigma_t) - Sigma_s^T) phi = chi (the mean chi of the fissile
 * materials for one that does not fission, 1/G if none does; |phi| floored at 1e-30),
 * then Sigma_t, Sigma_a = Sigma_t - sum_g' Sigma_s,g->g' and nuSigma_f. MOC_EINVAL for
 * null pointers, M <= 0 or G outside 1..32. */
int cnn_material_features(const double *sigma_t, const double *sigma_s, const double *nu_sigma_f, const double *chi,
                          int32_t M, int32_t G, float *features, void *stream);

/* Rasterise: out[p][c] = bf16(table[idx[p]][c]) for c < C, 0 for C <= c < Cp
 * (idx [npix] int32 in [0, rows), table FP32 [rows][C]). */
int cnn_gather_rows(const float *table, const int32_t *idx, int64_t npix, int32_t C, int32_t Cp,
                    uint16_t *out, void *stream);

/* out[p][c] = log(table[idx[p]][c]) for c < C, 0 for C <= c < Cp (table FP64 [rows][C],
 * positive; out FP32 [npix][Cp]): training targets from a converged scalar flux. */
int cnn_gather_log(const double *table, const int32_t *idx, int64_t npix, int32_t C, int32_t Cp,
                   float *out, void *stream);

/* Training targets as a shape: for each of n_images images FP32 [npix][Cp] (in place),
 * subtract the mean over its pixels and channels [0, C) from those entries. The solver
 * rescales any guess, so only the shape of log(phi) is worth learning. */
int cnn_center(float *img, int64_t n_images, int64_t npix, int32_t C, int32_t Cp, void *stream);

/* Square-image symmetry op in 0..7 (identity, rotations by 90, 180 and 270 degrees,
 * transpose, the two mirrors, anti-transpose): y [N][S][S][C] BF16 = x transformed
 * (y[r][c] = x[source_op(r, c)]). x and y must not overlap. */
int cnn_d4_transform(const uint16_t *x, int32_t N, int32_t S, int32_t C, int32_t op, uint16_t *y, void *stream);

/* acc [S][S][Cs] FP32, channels [0, C) += weight * (y transformed back by the inverse of
 * op), y [S][S][Cs] FP32 the network's output on the image transformed by op: averaging
 * the outputs of all 8 ops gives a prediction that respects the square's symmetry. */
int cnn_d4_accumulate(const float *y, int32_t S, int32_t Cs, int32_t C, int32_t op, float weight, float *acc,
                      void *stream);

/* De-rasterise: for each of n points with pixel coordinates (u, v) (x then y, pixel
 * centres at integers), bilinear interpolation of img FP32 [H][W][Cs] channels [0, C),
 * clamped at the border; out FP64 [n][C] = exp(value) if apply_exp else value. */
int cnn_bilinear_sample(const float *img, int32_t H, int32_t W, int32_t Cs, int32_t C, const float *uv,
                        int64_t n, int32_t apply_exp, double *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CNN_H */
