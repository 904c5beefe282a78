/* sg_cnn.h -- C ABI of the learned gradient preconditioner in libseisgrad.
 *
 * The paper has no network.  Its Limitations section calls ill-conditioning
 * intrinsic to the inversion and notes that conditioning techniques can be
 * applied within the framework; this part is one such technique, of the
 * project's own design.  What it preconditions is the
 * gradient of the paper's method (Method section: the misfit after Eq. (1),
 * its gradient by the adjoint Eqs. (4)-(5)), used by plain gradient-descent
 * inversion.  The network is fixed:
 *
 *     x1 = relu(c1(g)),  a2 = relu(c2(x1)),  x2 = relu(c3(a2) + x1),
 *     a4 = relu(c4(x2)), x3 = relu(c5(a4) + x2),  p = -g + c6(x3),
 *
 * with 3x3 cross-correlations and one cell of zero padding; c1: 1 -> 32
 * channels, c2..c5: 32 -> 32, c6: 32 -> 1.  The parameters are one FP32
 * vector of CNN_NPARAMS numbers, layer by layer c1..c6, each layer's weights
 * as [Cout][3][3][Cin] followed by its Cout biases.
 *
 * Precision: images (g, p, targets, masks) are FP32 [n][h][w]; the hidden
 * activations x1, a2, x2, a4, x3 and their back-propagated gradients are BF16
 * (round to nearest even) channels-last [n][h][w][32]; c2..c5 run on BF16
 * operands with FP32 accumulation on the matrix cores; c1 and c6 run in FP32.
 * Parameter gradients are reduced in a fixed order, so every call is bitwise
 * reproducible.
 *
 * Conventions: all pointers are device pointers, 16-byte aligned where they
 * address BF16 activations; calls are asynchronous on `stream` (NULL = the
 * null stream); they return SG_OK or a negative SG_E* code (seisgrad.h) with
 * a message in last_error().  Image extents must be positive with n h w
 * below 2^29 pixels (SG_EINVAL otherwise).  The library allocates nothing: scratch comes
 * from the caller's workspace.  Calls that share a workspace must not overlap.
 */
#ifndef SG_CNN_H
#define SG_CNN_H

#include "seisgrad.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CNN_CHANNELS 32
#define CNN_NPARAMS 37601

/* Bytes of workspace for images of n x h x w: BF16 weight copies, the five
 * saved activations, three gradient buffers and reduction partials. */
SG_API size_t cnn_workspace_bytes(int32_t n, int32_t h, int32_t w);

/* p = -g + N(g) for n images g [n][h][w] (FP32).  Saves the activations in
 * `ws` for a following cnn_backward on the same images and parameters. */
SG_API int cnn_forward(const float *params, const float *g, int32_t n, int32_t h, int32_t w,
                       float *p, void *ws, size_t ws_bytes, sg_stream_t stream);

/* grad = d(sum(dp * p))/d(params) (FP32, CNN_NPARAMS, overwritten) for the
 * images, parameters and workspace of the last cnn_forward (not checked). */
SG_API int cnn_backward(const float *params, const float *g, const float *dp, int32_t n,
                        int32_t h, int32_t w, float *grad, void *ws, size_t ws_bytes,
                        sg_stream_t stream);

/* Masked mean squared error over `count` cells: L = sum(mask (p - t)^2) /
 * sum(mask), accumulated in FP64 into *L_dev; dp = dL/dp (FP32, may be NULL).
 * mask holds 0 or 1; an all-zero mask gives L = 0 and dp = 0.  Uses the
 * reduction area of a workspace of at least cnn_workspace_bytes(1, 1, 1). */
SG_API int cnn_loss(const float *p, const float *t, const float *mask, int64_t count,
                    double *L_dev, float *dp, void *ws, size_t ws_bytes, sg_stream_t stream);

/* One Adam step (step counts from 1) on n parameters, FP32 state m, v. */
SG_API int cnn_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                    float beta1, float beta2, float eps, int32_t step, sg_stream_t stream);

/* Packs nfields slots of the fields a, b [nsrc][fh][fw] into patches of
 * 2 x 2 frames of frame x frame cells: slot s (field order[s], or s when
 * order is NULL) sits in the top-left corner of frame s % 4 (row-major) of
 * patch s / 4; everything else is zero.  An order entry outside [0, nsrc)
 * gives an all-zero slot with mask 0.  The packed value is a - b (b may be NULL), times
 * 1/RMS of that field when normalise != 0 (FP64 reduction; inv_rms[s]
 * receives the factor, 0 for an all-zero field).  mask (may be NULL) gets 1
 * on the field cells and 0 elsewhere.  patches and mask are
 * [ceil(nfields/4)][2 frame][2 frame].  Requires fh, fw <= frame. */
SG_API int cnn_pack(const float *a, const float *b, int32_t nsrc, const int32_t *order, int32_t nfields,
                    int32_t fh, int32_t fw, int32_t frame, int32_t normalise, double *inv_rms,
                    float *patches, float *mask, sg_stream_t stream);

/* Inverse of cnn_pack's placement: fields[s] = the fh x fw corner of slot s. */
SG_API int cnn_unpack(const float *patches, int32_t nfields, int32_t fh, int32_t fw, int32_t frame,
                      float *fields, sg_stream_t stream);

/* One 32 -> 32 channel 3x3 layer on BF16 channels-last images x [n][h][w][32]
 * with BF16 weights wgt [32][3][3][32]:  v = sum + bias (may be NULL) + res
 * (may be NULL, BF16 like x); v = max(v, 0) if relu; v = 0 where gate <= 0
 * (gate may be NULL, BF16 like x).  y gets v in BF16, y32 (may be NULL) in
 * FP32.  This is the forward of c2..c5 and, with the weights flipped and
 * transposed, their input gradient.  x, wgt, res, gate, y and y32 must be
 * 16-byte aligned (SG_EINVAL otherwise). */
SG_API int cnn_conv3x3(const uint16_t *x, int32_t n, int32_t h, int32_t w, const uint16_t *wgt,
                       const float *bias, const uint16_t *res, const uint16_t *gate, int32_t relu,
                       uint16_t *y, float *y32, sg_stream_t stream);

/* Weight and bias gradient of one 32 -> 32 layer: dw[co][ky][kx][ci] =
 * sum over pixels of dy[pix][co] x[pix + (ky-1, kx-1)][ci], then db[co] =
 * sum of dy[pix][co]; dw gets 9216 + 32 FP32 numbers in that order. */
SG_API int cnn_conv3x3_wgrad(const uint16_t *dy, const uint16_t *x, int32_t n, int32_t h, int32_t w,
                             float *dw, void *ws, size_t ws_bytes, sg_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SG_CNN_H */
