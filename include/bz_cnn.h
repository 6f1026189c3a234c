/*
 * bz_cnn.h -- C ABI of the matrix-core convolutions of libbz's learned curve
 * initialiser: a small convolutional network that maps an image patch to the
 * initial parameters of the curves of that patch (a project-defined
 * component; the paper initialises curves at random, Sec. 3.5, which stays
 * the fallback).
 *
 * Layouts: activations NHWC (channels fastest); filters [k][r][r][c] (output
 * channel, filter row, filter column, input channel).  BF16 operands are
 * passed as uint16_t bit patterns (bfloat16: the high half of an IEEE
 * float32, round to nearest even).  Products are accumulated in FP32 on the
 * matrix cores (v_mfma_f32_16x16x32_bf16).
 *
 * Conventions of bz.h apply: device pointers owned by the caller, no
 * allocation, asynchronous on the caller's stream, argument errors on the
 * host before any launch.
 */
#ifndef BZ_CNN_H
#define BZ_CNN_H

#include "bz.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One convolution: input [n][h][w][c], output [n][ho][wo][k] with
 * ho = (h + 2 pad - r) / stride + 1 (same for wo).  A fully connected layer
 * is the case h = w = r = 1. */
typedef struct {
    int32_t n, h, w, c;
    int32_t k;
    int32_t r;               /* 1 or 3 */
    int32_t stride, pad;     /* stride 1..4, 0 <= pad < r */
    int32_t ho, wo;          /* set by bz_conv_shape */
} bz_conv;

/* Host: validate the sizes and set ho, wo.  BZ_ERR_ARG for non-positive
 * sizes, an empty output or a bad filter; BZ_ERR_UNSUPPORTED from 2^30
 * elements per tensor. */
bz_status bz_conv_shape(bz_conv *cv);

/* y[m][o] = bias[o] + sum_{dy, dx, i} x[pixel m shifted by (dy, dx)][i] w[o][dy][dx][i]
 * (zero padding), then max(0, .) if relu.  y (FP32, may be NULL) and y_bf16
 * (may be NULL, not both) receive the result; bias may be NULL (0). */
bz_status bz_conv_fwd(const bz_conv *cv, const uint16_t *x, const uint16_t *w,
                      const float *bias, int32_t relu, float *y, uint16_t *y_bf16,
                      hipStream_t stream);

/* Gradient with respect to the input: dx = w^T * dy, the adjoint of
 * bz_conv_fwd's sum (dy rounded to BF16 as it enters the matrix cores).
 * x_mask (may be NULL): the layer's BF16 input; where it is <= 0 the
 * gradient is zeroed, which applies the derivative of the ReLU that produced
 * it.  dx: FP32 [n][h][w][c], overwritten. */
bz_status bz_conv_bwd_data(const bz_conv *cv, const float *dy, const uint16_t *w,
                           const uint16_t *x_mask, float *dx, hipStream_t stream);

/* Gradients with respect to the filters and the bias: dw = sum over output
 * pixels of dy x^T (dy rounded to BF16), db = sum of dy (FP32).  dw: FP32
 * [k][r][r][c], db: [k] or NULL; both overwritten.  Sums over pixels use
 * float atomics (run-to-run differences in the last bits). */
bz_status bz_conv_bwd_weight(const bz_conv *cv, const float *dy, const uint16_t *x,
                             float *dw, float *db, hipStream_t stream);

/* src FP32 -> dst BF16 (round to nearest even), n elements. */
bz_status bz_f32_to_bf16(const float *src, uint16_t *dst, int64_t n, hipStream_t stream);

/* Patches of an image for the network: image planar [3][height][width] FP32;
 * patch p has its top-left pixel at (xy[2p], xy[2p+1]) and side `side`;
 * pixels outside the image read `fill`.  out: BF16 NHWC [n_patch][side][side][3]. */
bz_status bz_extract_patches(const float *image, int32_t width, int32_t height,
                             const int32_t *xy, int32_t n_patch, int32_t side, float fill,
                             uint16_t *out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* BZ_CNN_H */
