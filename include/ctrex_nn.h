/*
 * ctrex_nn.h — C ABI of the learned-correction kernels (3D U-Net).
 *
 * The paper names learned components acting as correction terms between
 * physics-based operator applications as the natural extension of its
 * operator framework (Sec. 5); this library provides the kernels of such a
 * correction: a 3D U-Net applied to the volume between unrolled SIRT
 * iterations of Eq. (1), trained and run on the GPU by these kernels.
 *
 * Conventions:
 *  - Activations are BF16, channels-last: element (z, y, x, c) of a tensor
 *    with channel stride `cs` and channel offset `off` sits at
 *    ((z * H + y) * W + x) * cs + off + c.  A stride larger than the channel
 *    count lets a layer read or write a slice of a wider tensor.  The
 *    decoder's skip concatenations are never stored: ctrex_nn_conv3_cat
 *    reads the two tensors and writes the two gradients directly (a stored
 *    concatenation costs its producers half-record writes, which the memory
 *    system turns into read-modify-writes).  Tensors of 16 or more
 *    channels are read 8 channels at a time (16-byte loads): their stride and
 *    offset must be multiples of 8 (CTREX_ESHAPE otherwise).  Volumes D x H x W need
 *    D * H * W to be a multiple of 64 and, for the 2x pooling and up-sampling,
 *    even sides.
 *  - Convolution weights are packed BF16 `[taps][cout][cin]` (cin fastest);
 *    3x3x3 taps are ordered (dz, dy, dx) with dx fastest, zero padding of 1.
 *    ctrex_nn_pack_conv3 builds the forward packing from FP32 master weights
 *    `[cout][cin][27]`, and the packing of the data gradient (taps mirrored,
 *    in/out channels swapped).  Up-sampling weights (2x2x2, stride 2) are FP32
 *    `[cin][cout][8]` (torch ConvTranspose3d order), packed as BF16
 *    `[8][cout][cin]` and, for the data gradient, `[8][cin][cout]`.
 *  - Arithmetic: BF16 x BF16 products accumulate in FP32 on the matrix cores
 *    (v_mfma_f32_16x16x32_bf16); biases, losses and optimizer state are FP32.
 *  - Channel counts: cin in {1, 16, 32, 64}, cout in {16, 32, 64} (the
 *    3-level 16/32/64 U-Net); other values return CTREX_ESHAPE.
 *  - All calls are asynchronous on `stream` (a hipStream_t, NULL = null
 *    stream) unless stated; pointers are device memory owned by the caller;
 *    statuses and ctrex_last_error() as in ctrex.h.
 *  - The weight-gradient, head-gradient and loss calls keep per-chunk partial
 *    sums in the device scratch attached to the context with
 *    ctrex_set_scratch; ctrex_nn_scratch_bytes gives the size one layer
 *    needs.  The library allocates none itself.
 */
#ifndef CTREX_NN_H
#define CTREX_NN_H

#include "ctrex.h"

#ifdef __cplusplus
extern "C" {
#endif

#define CTREX_NN_RELU 1u       /* apply max(., 0) in the epilogue */
#define CTREX_NN_ACCUMULATE 2u /* add into the output instead of overwriting */
#define CTREX_NN_OUT_F32 4u    /* output tensor is FP32 (default BF16) */

/*
 * Bytes of attached scratch (ctrex_set_scratch) that the learned-correction
 * calls need for a layer of cin -> cout channels over n_vox voxels (the
 * input volume of a weight gradient): the maximum over the weight and bias
 * gradients of the convolution and the transposed convolution, the head's
 * gradient and the loss.  A network needs the maximum over its layers.
 */
CTREX_API int ctrex_nn_scratch_bytes(int32_t cin, int32_t cout, int64_t n_vox, size_t *bytes);

/*
 * out = act(bias + conv3x3x3(in, w)) over a D x H x W volume (stride 1, zero
 * padding 1).  `wt` is a packed BF16 [27][cout][cin] weight tensor, `bias` FP32
 * [cout] or NULL.  With CTREX_NN_ACCUMULATE the result (after the activation)
 * is added to `out`.  The data gradient of a convolution is this call with
 * the dgrad packing of its weights (cin and cout swapped), no bias, no ReLU.
 */
CTREX_API int ctrex_nn_conv3(ctrex_ctx *ctx, const void *in, int32_t in_cs, int32_t in_off,
                             int32_t cin, const void *wt, const float *bias, void *out,
                             int32_t out_cs, int32_t out_off, int32_t cout, int32_t D, int32_t H,
                             int32_t W, uint32_t flags, void *stream);

/*
 * Weight and bias gradients of ctrex_nn_conv3: dw[co][ci][tap] (FP32, same
 * order as the master weights) = sum over voxels of dout[v][co] *
 * in[v + tap][ci]; dbias[co] = sum over voxels of dout[v][co] (NULL skips).
 * Results overwrite dw / dbias; sums are formed in FP32 per chunk of voxels
 * and combined in a fixed order in FP64 (deterministic).  The per-chunk
 * partial sums go to the scratch attached with ctrex_set_scratch (sized by
 * ctrex_nn_scratch_bytes; CTREX_EWORKSPACE when too small).
 */
CTREX_API int ctrex_nn_conv3_wgrad(ctrex_ctx *ctx, const void *in, int32_t in_cs, int32_t in_off,
                                   int32_t cin, const void *dout, int32_t dout_cs,
                                   int32_t dout_off, int32_t cout, int32_t D, int32_t H, int32_t W,
                                   float *dw, float *dbias, void *stream);

/*
 * ctrex_nn_conv3 over the channel concatenation of two tensors, written to
 * two tensors: the U-Net decoder's convolution of [up-sampled features |
 * skip features] and, with the dgrad packing, its data gradient split back
 * into the two parts.  Input channels [0, ca) are in_a's channels a_off ..
 * a_off + ca - 1 (stride a_cs), input channels [ca, ca + cb) in_b's channels
 * b_off .. (stride b_cs); output channels [0, oa) go to out_a (stride oa_cs,
 * offset oa_off), [oa, oa + ob) to out_b.  cb = 0 ignores in_b, ob = 0
 * ignores out_b (then this is ctrex_nn_conv3).  `gate` (NULL = none; channel
 * stride g_cs and offset g_off, multiples of 8) zeroes output channel co of
 * voxel v where gate[v][g_off + co] <= 0 (or NaN), before the activation and
 * accumulation: with gate = the forward ReLU output, a data-gradient
 * convolution writes the gradient at that layer's pre-activation (the ReLU
 * backward folded in).  A two-tensor input (cb > 0)
 * is supported for (ca + cb, oa + ob) = (32, 16) or (64, 32) with ca a
 * multiple of 8; a two-tensor output (ob > 0) needs cin >= 16 and oa a
 * multiple of 16; a gate needs cin >= 16; other shapes as ctrex_nn_conv3,
 * CTREX_ESHAPE otherwise.
 * Same flags, packing, arithmetic and status behaviour as ctrex_nn_conv3.
 */
CTREX_API int ctrex_nn_conv3_cat(ctrex_ctx *ctx, const void *in_a, int32_t a_cs, int32_t a_off,
                                 int32_t ca, const void *in_b, int32_t b_cs, int32_t b_off,
                                 int32_t cb, const void *wt, const float *bias, void *out_a,
                                 int32_t oa_cs, int32_t oa_off, int32_t oa, void *out_b,
                                 int32_t ob_cs, int32_t ob_off, int32_t ob, const void *gate,
                                 int32_t g_cs, int32_t g_off, int32_t D, int32_t H, int32_t W,
                                 uint32_t flags, void *stream);

/*
 * ctrex_nn_conv3_wgrad with the input the channel concatenation of in_a
 * (ca channels) and in_b (cb channels, 0 = none), both in {16, 32, 64} with
 * ca + cb <= 64: dw[co][ci][tap] over ci < ca + cb in concatenation order.
 * Scratch, determinism and statuses as ctrex_nn_conv3_wgrad.
 */
CTREX_API int ctrex_nn_conv3_wgrad_cat(ctrex_ctx *ctx, const void *in_a, int32_t a_cs,
                                       int32_t a_off, int32_t ca, const void *in_b, int32_t b_cs,
                                       int32_t b_off, int32_t cb, const void *dout,
                                       int32_t dout_cs, int32_t dout_off, int32_t cout, int32_t D,
                                       int32_t H, int32_t W, float *dw, float *dbias,
                                       void *stream);

/*
 * The last decoder convolution with the head folded in: a = BF16(ReLU(bias +
 * conv3x3x3(in, w))) for 16 -> 16 channels (packing as ctrex_nn_conv3), then
 * out[v] = x[v] + m[v] out_scale (hb[0] + sum_c h[c] a[v][c]) as
 * ctrex_nn_head computes it (the 16 products are summed in another order, so
 * results may differ from the two calls in the last bits).  `act` (BF16,
 * channel stride act_cs, offset act_off; NULL = not stored) receives a, which
 * only training needs; `mask` as in ctrex_nn_head.
 */
CTREX_API int ctrex_nn_conv3_head(ctrex_ctx *ctx, const void *in, int32_t in_cs, int32_t in_off,
                                  const void *wt, const float *bias, void *act, int32_t act_cs,
                                  int32_t act_off, const float *h, const float *hb,
                                  const float *x, float out_scale, const float *mask, float *out,
                                  int32_t D, int32_t H, int32_t W, void *stream);

/*
 * 2x2x2 stride-2 transposed convolution (up-sampling): the input is
 * D x H x W, the output 2D x 2H x 2W; out[2i + a][co] = bias[co] +
 * sum_ci in[i][ci] w[a][co][ci], `wt` packed BF16 [8][cout][cin].
 */
CTREX_API int ctrex_nn_upconv2(ctrex_ctx *ctx, const void *in, int32_t in_cs, int32_t in_off,
                               int32_t cin, const void *wt, const float *bias, void *out,
                               int32_t out_cs, int32_t out_off, int32_t cout, int32_t D,
                               int32_t H, int32_t W, uint32_t flags, void *stream);

/*
 * Data gradient of ctrex_nn_upconv2: din[i][ci] = sum_a sum_co
 * dout[2i + a][co] w[a][co][ci] (`wt_d` packed BF16 [8][cin][cout]); D, H, W
 * are the sizes of `din`.
 */
CTREX_API int ctrex_nn_upconv2_dgrad(ctrex_ctx *ctx, const void *dout, int32_t dout_cs,
                                     int32_t dout_off, int32_t cout, const void *wt_d, void *din,
                                     int32_t din_cs, int32_t din_off, int32_t cin, int32_t D,
                                     int32_t H, int32_t W, uint32_t flags, void *stream);

/*
 * Weight and bias gradients of ctrex_nn_upconv2: dw[ci][co][a] (FP32, torch
 * ConvTranspose3d order) and dbias[co] (NULL skips); D, H, W are the input
 * sizes.  Deterministic, like ctrex_nn_conv3_wgrad.
 */
CTREX_API int ctrex_nn_upconv2_wgrad(ctrex_ctx *ctx, const void *in, int32_t in_cs,
                                     int32_t in_off, int32_t cin, const void *dout,
                                     int32_t dout_cs, int32_t dout_off, int32_t cout, int32_t D,
                                     int32_t H, int32_t W, float *dw, float *dbias, void *stream);

/* 2x2x2 max pooling: out[i][c] = max_a in[2i + a][c]; D, H, W are the input
 * sizes; `out` is dense (channel stride = c). */
CTREX_API int ctrex_nn_maxpool2(ctrex_ctx *ctx, const void *in, int32_t in_cs, int32_t in_off,
                                int32_t c, void *out, int32_t D, int32_t H, int32_t W,
                                void *stream);

/* Backward of ctrex_nn_maxpool2: din[2i + a][c] += dout[i][c] for the first
 * (in x, y, z order) maximum of each window; `din` shares the layout of `in`. */
CTREX_API int ctrex_nn_maxpool2_backward(ctrex_ctx *ctx, const void *in, int32_t in_cs,
                                         int32_t in_off, int32_t c, const void *dout, void *din,
                                         int32_t D, int32_t H, int32_t W, void *stream);

/* ctrex_nn_maxpool2_backward followed by ctrex_nn_relu_backward with y = in
 * over the whole slice, in one pass (`in` is a ReLU output): din[v][c] = 0
 * where in[v][c] <= 0 (or NaN), otherwise din plus the pooled gradient as
 * above.  Only the window maxima's din is read. */
CTREX_API int ctrex_nn_maxpool2_relu_backward(ctrex_ctx *ctx, const void *in, int32_t in_cs,
                                              int32_t in_off, int32_t c, const void *dout,
                                              void *din, int32_t D, int32_t H, int32_t W,
                                              void *stream);

/* ReLU backward in place: g[v][c] = 0 where y[v][c] <= 0 (y, g share the
 * channel stride/offset layout; n_vox voxels of c channels). */
CTREX_API int ctrex_nn_relu_backward(ctrex_ctx *ctx, const void *y, void *g, int32_t cs,
                                     int32_t off, int32_t c, int64_t n_vox, void *stream);

/* Network input: xb[v] = BF16(scale x[v]) (round to nearest even); x FP32.
 * The scale brings volumes stored in small physical units (attenuation per
 * volume width) to the O(1) range the network's biases work in. */
CTREX_API int ctrex_nn_input(ctrex_ctx *ctx, const float *x, float scale, void *xb, int64_t n_vox,
                             void *stream);

/* Head and residual: out[v] = x[v] + m[v] out_scale (b + sum_c h[c] act[v][c])
 * (x, out FP32, act BF16 dense with c channels, h FP32 [c], b FP32 [1]);
 * out_scale = 1 / the input scale maps the correction back to x's units;
 * `mask` (FP32 [n_vox], NULL = all ones) confines the correction, e.g. to the
 * scanned field of view. */
CTREX_API int ctrex_nn_head(ctrex_ctx *ctx, const void *act, int32_t c, const float *h,
                            const float *b, const float *x, float out_scale, const float *mask,
                            float *out, int64_t n_vox, void *stream);

/* Backward of ctrex_nn_head: with d = m out_scale dout, dact[v][c] = d[v] h[c]
 * (BF16), dh[c] = sum_v d[v] act[v][c], db = sum_v d[v] (FP32, deterministic). */
CTREX_API int ctrex_nn_head_backward(ctrex_ctx *ctx, const void *act, int32_t c, const float *h,
                                     float out_scale, const float *mask, const float *dout,
                                     void *dact, float *dh, float *db, int64_t n_vox,
                                     void *stream);

/* ctrex_nn_head_backward with dact also multiplied by the ReLU derivative at
 * act (dact = 0 where act <= 0 or NaN): the gradient at the pre-activation of
 * the layer whose ReLU output the head reads, in one pass. */
CTREX_API int ctrex_nn_head_relu_backward(ctrex_ctx *ctx, const void *act, int32_t c,
                                          const float *h, float out_scale, const float *mask,
                                          const float *dout, void *dact, float *dh, float *db,
                                          int64_t n_vox, void *stream);

/* Weighted mean squared error over n values: *loss (host, optional; waits)
 * = weight sum (a - t)^2 / n with the sum in FP64, grad (optional) =
 * 2 weight (a - t) / n.  A weight of s^2 measures the error in the units of a
 * network that reads s x, which keeps weight gradients well above Adam's
 * epsilon when volumes are stored in small units. */
CTREX_API int ctrex_nn_mse(ctrex_ctx *ctx, const float *a, const float *t, int64_t n,
                           float weight, double *loss, float *grad, void *stream);

/* One Adam step over n FP32 parameters (bias-corrected, step >= 1). */
CTREX_API int ctrex_nn_adam(ctrex_ctx *ctx, float *param, const float *grad, float *m, float *v,
                            int64_t n, float lr, float beta1, float beta2, float eps,
                            int32_t step, void *stream);

/* Pack FP32 master weights [cout][cin][27] into BF16 forward [27][cout][cin]
 * (`wt`, optional) and data-gradient [27][cin][cout] with mirrored taps
 * (`wt_d`, optional). */
CTREX_API int ctrex_nn_pack_conv3(ctrex_ctx *ctx, const float *w, int32_t cout, int32_t cin,
                                  void *wt, void *wt_d, void *stream);

/* Pack FP32 up-sampling weights [cin][cout][8] into BF16 [8][cout][cin]
 * (`wt`, optional) and [8][cin][cout] (`wt_d`, optional). */
CTREX_API int ctrex_nn_pack_upconv2(ctrex_ctx *ctx, const float *w, int32_t cin, int32_t cout,
                                    void *wt, void *wt_d, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CTREX_NN_H */
