// C ABI of the learned-correction kernels (include/ctrex_nn.h): host-side
// validation, scratch management and launches.

#include "../../include/ctrex_nn.h"

#include <algorithm>
#include <cmath>

#include "ctrex_ctx.h"
#include "ctrex_internal.h"

namespace ctrex {
namespace nn {
hipError_t launch_conv3(const void *in, int in_cs, int in_off, int cin_a, const void *in2,
                        int in2_cs, int in2_off, int cin_b, const void *wt, const float *bias,
                        void *out, int out_cs, int out_off, int cout_a, void *out2, int out2_cs,
                        int out2_off, int cout_b, const void *gate, int gate_cs, int gate_off,
                        int D, int H, int W, bool relu, bool acc, bool out_f32, hipStream_t s);
hipError_t launch_conv3_head(const void *in, int in_cs, int in_off, const void *wt,
                             const float *bias, void *act, int act_cs, int act_off, const float *h,
                             const float *hb, const float *x, float scale, const float *mask,
                             float *out, int D, int H, int W, hipStream_t s);
size_t conv3_wgrad_scratch(int cin, int cout, long long nvox);
hipError_t launch_conv3_wgrad(const void *in, int in_cs, int in_off, int cin_a, const void *in2,
                              int in2_cs, int in2_off, int cin_b, const void *dout, int dout_cs,
                              int dout_off, int cout, int D, int H, int W, float *dw,
                              float *dbias, float *scratch, hipStream_t s);
size_t channel_sum_scratch(int c);
hipError_t launch_channel_sum(const void *x, int cs, int off, int c, long long nvox, float *out,
                              double *scratch, hipStream_t s);
hipError_t launch_upconv2(const void *in, int in_cs, int in_off, int cin, const void *wt,
                          const float *bias, void *out, int out_cs, int out_off, int cout, int D,
                          int H, int W, bool acc, bool out_f32, hipStream_t s);
hipError_t launch_upconv2_dgrad(const void *dout, int dout_cs, int dout_off, int cout,
                                const void *wd, void *din, int din_cs, int din_off, int cin, int D,
                                int H, int W, bool acc, hipStream_t s);
size_t upconv2_wgrad_scratch(int cin, int cout, long long nvox);
hipError_t launch_upconv2_wgrad(const void *in, int in_cs, int in_off, int cin, const void *dout,
                                int dout_cs, int dout_off, int cout, int D, int H, int W,
                                float *dw, float *scratch, hipStream_t s);
hipError_t launch_maxpool2(const void *in, int in_cs, int in_off, int c, void *out, int D, int H,
                           int W, hipStream_t s);
hipError_t launch_maxpool2_bwd(const void *in, int in_cs, int in_off, int c, const void *dout,
                               void *din, int D, int H, int W, bool relu, hipStream_t s);
hipError_t launch_relu_bwd(const void *y, void *g, int cs, int off, int c, long long nvox,
                           hipStream_t s);
hipError_t launch_head(const void *act, int c, const float *h, const float *b, const float *x,
                       float scale, const float *mask, float *out, long long n, hipStream_t s);
hipError_t launch_scale_bf16(const float *x, float scale, void *xb, long long n, hipStream_t s);
size_t head_bwd_scratch(int c);
hipError_t launch_head_bwd(const void *act, int c, const float *h, float scale, const float *mask,
                           const float *dout, void *dact, float *dh, float *db, long long n,
                           bool relu, double *scratch, hipStream_t s);
hipError_t launch_mse(const float *a, const float *t, long long n, float weight, float *grad,
                      double *partial, int blocks, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);
hipError_t launch_pack(const float *w, int cout, int cin, int taps, bool mirror, void *wt,
                       void *wt_d, bool in_major, hipStream_t s);
}  // namespace nn
}  // namespace ctrex

using namespace ctrex;

namespace {

constexpr int kMseBlocks = 1024;   // per-block partials of ctrex_nn_mse

bool chan_ok(int c) { return c == 16 || c == 32 || c == 64; }

int check_vol(ctrex_ctx *c, int D, int H, int W, bool even) {
    if (D < 1 || H < 1 || W < 1) return fail(c, CTREX_ESHAPE, "volume sides must be >= 1");
    const long long n = static_cast<long long>(D) * H * W;
    if (n % 64 != 0) return fail(c, CTREX_ESHAPE, "D*H*W = %lld is not a multiple of 64", n);
    if (n * 64 >= (1ll << 40)) return fail(c, CTREX_ESHAPE, "volume too large");
    if (even && (D % 2 || H % 2 || W % 2)) return fail(c, CTREX_ESHAPE, "sides must be even");
    return CTREX_OK;
}

// A channels-last tensor slice: cs >= off + c; 16-byte loads need cs, off % 8 == 0.
int check_slice(ctrex_ctx *c, const char *what, const void *p, int cs, int off, int ch,
                bool vec_loads) {
    if (!p) return fail(c, CTREX_EINVAL, "%s is NULL", what);
    if (off < 0 || cs < off + ch) return fail(c, CTREX_ESHAPE, "%s: channel stride %d < offset %d + %d",
                                              what, cs, off, ch);
    if (vec_loads && (cs % 8 || off % 8))
        return fail(c, CTREX_ESHAPE, "%s: channel stride and offset must be multiples of 8", what);
    return CTREX_OK;
}

int begin(ctrex_ctx *c) {
    if (!c) return CTREX_EINVAL;
    CTREX_HIP(c, hipSetDevice(c->device));
    return CTREX_OK;
}

int maxpool2_backward(ctrex_ctx *c, const void *in, int32_t in_cs, int32_t in_off, int32_t ch,
                      const void *dout, void *din, int32_t D, int32_t H, int32_t W, bool relu,
                      void *stream) {
    int st = begin(c);
    if (st) return st;
    if (ch < 1) return fail(c, CTREX_ESHAPE, "c must be >= 1");
    if (D < 2 || H < 2 || W < 2 || D % 2 || H % 2 || W % 2)
        return fail(c, CTREX_ESHAPE, "pooling needs even sides >= 2");
    if ((st = check_slice(c, "in", in, in_cs, in_off, ch, false))) return st;
    if (!dout || !din) return fail(c, CTREX_EINVAL, "dout and din must be device pointers");
    CTREX_HIP(c, nn::launch_maxpool2_bwd(in, in_cs, in_off, ch, dout, din, D, H, W, relu,
                                         static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int head_backward(ctrex_ctx *c, const void *act, int32_t ch, const float *h, float out_scale,
                  const float *mask, const float *dout, void *dact, float *dh, float *db,
                  int64_t n_vox, bool relu, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!act || !h || !dout || !dact) return fail(c, CTREX_EINVAL, "NULL pointer");
    if (ch != 16 || n_vox < 1) return fail(c, CTREX_ESHAPE, "the head takes 16 channels");
    if (!std::isfinite(out_scale)) return fail(c, CTREX_EINVAL, "out_scale must be finite");
    void *scr;
    if ((st = ctx_scratch(c, nn::head_bwd_scratch(ch), &scr))) return st;
    CTREX_HIP(c, nn::launch_head_bwd(act, ch, h, out_scale, mask, dout, dact, dh, db, n_vox, relu,
                                     static_cast<double *>(scr), static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}
}  // namespace

extern "C" {

int ctrex_nn_conv3(ctrex_ctx *c, const void *in, int32_t in_cs, int32_t in_off, int32_t cin,
                   const void *wt, const float *bias, void *out, int32_t out_cs, int32_t out_off,
                   int32_t cout, int32_t D, int32_t H, int32_t W, uint32_t flags, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!(cin == 1 || chan_ok(cin)) || !chan_ok(cout))
        return fail(c, CTREX_ESHAPE, "unsupported channels %d -> %d", cin, cout);
    if (flags & ~(CTREX_NN_RELU | CTREX_NN_ACCUMULATE | CTREX_NN_OUT_F32))
        return fail(c, CTREX_EINVAL, "unknown flags");
    if ((st = check_vol(c, D, H, W, false))) return st;
    if ((st = check_slice(c, "in", in, in_cs, in_off, cin, cin > 1))) return st;
    if ((st = check_slice(c, "out", out, out_cs, out_off, cout, false))) return st;
    if (!wt) return fail(c, CTREX_EINVAL, "wt is NULL");
    CTREX_HIP(c, nn::launch_conv3(in, in_cs, in_off, cin, nullptr, 0, 0, 0, wt, bias, out, out_cs,
                                  out_off, cout, nullptr, 0, 0, 0, nullptr, 0, 0, D, H, W,
                                  flags & CTREX_NN_RELU, flags & CTREX_NN_ACCUMULATE,
                                  flags & CTREX_NN_OUT_F32, static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_conv3_cat(ctrex_ctx *c, const void *in_a, int32_t a_cs, int32_t a_off, int32_t ca,
                       const void *in_b, int32_t b_cs, int32_t b_off, int32_t cb, const void *wt,
                       const float *bias, void *out_a, int32_t oa_cs, int32_t oa_off, int32_t oa,
                       void *out_b, int32_t ob_cs, int32_t ob_off, int32_t ob, const void *gate,
                       int32_t g_cs, int32_t g_off, int32_t D, int32_t H, int32_t W,
                       uint32_t flags, void *stream) {
    int st = begin(c);
    if (st) return st;
    const int cin = ca + cb, cout = oa + ob;
    if (ca < 1 || cb < 0 || oa < 1 || ob < 0 || !(cin == 1 || chan_ok(cin)) || !chan_ok(cout))
        return fail(c, CTREX_ESHAPE, "unsupported channels %d + %d -> %d + %d", ca, cb, oa, ob);
    if (cb > 0 && !((cin == 32 && cout == 16) || (cin == 64 && cout == 32)) )
        return fail(c, CTREX_ESHAPE, "a two-tensor input needs 32 -> 16 or 64 -> 32 channels");
    if (cb > 0 && ca % 8)
        return fail(c, CTREX_ESHAPE, "the first input's channel count must be a multiple of 8");
    if (ob > 0 && (oa % 16 || cin == 1))
        return fail(c, CTREX_ESHAPE, "a two-tensor output needs cin >= 16 and oa a multiple of 16");
    if (flags & ~(CTREX_NN_RELU | CTREX_NN_ACCUMULATE | CTREX_NN_OUT_F32))
        return fail(c, CTREX_EINVAL, "unknown flags");
    if ((st = check_vol(c, D, H, W, false))) return st;
    if ((st = check_slice(c, "in_a", in_a, a_cs, a_off, ca, cin > 1))) return st;
    if (cb > 0 && (st = check_slice(c, "in_b", in_b, b_cs, b_off, cb, true))) return st;
    if ((st = check_slice(c, "out_a", out_a, oa_cs, oa_off, oa, false))) return st;
    if (ob > 0 && (st = check_slice(c, "out_b", out_b, ob_cs, ob_off, ob, false))) return st;
    if (gate && cin == 1) return fail(c, CTREX_ESHAPE, "a gate needs cin >= 16");
    if (gate && (st = check_slice(c, "gate", gate, g_cs, g_off, cout, true))) return st;
    if (!wt) return fail(c, CTREX_EINVAL, "wt is NULL");
    CTREX_HIP(c, nn::launch_conv3(in_a, a_cs, a_off, ca, in_b, b_cs, b_off, cb, wt, bias, out_a,
                                  oa_cs, oa_off, oa, out_b, ob_cs, ob_off, ob, gate, g_cs, g_off,
                                  D, H, W,
                                  flags & CTREX_NN_RELU, flags & CTREX_NN_ACCUMULATE,
                                  flags & CTREX_NN_OUT_F32, static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_conv3_head(ctrex_ctx *c, const void *in, int32_t in_cs, int32_t in_off,
                        const void *wt, const float *bias, void *act, int32_t act_cs,
                        int32_t act_off, const float *h, const float *hb, const float *x,
                        float out_scale, const float *mask, float *out, int32_t D, int32_t H,
                        int32_t W, void *stream) {
    int st = begin(c);
    if (st) return st;
    if ((st = check_vol(c, D, H, W, false))) return st;
    if ((st = check_slice(c, "in", in, in_cs, in_off, 16, true))) return st;
    if (act && (st = check_slice(c, "act", act, act_cs, act_off, 16, false))) return st;
    if (!wt || !h || !hb || !x || !out) return fail(c, CTREX_EINVAL, "NULL pointer");
    if (!std::isfinite(out_scale)) return fail(c, CTREX_EINVAL, "out_scale must be finite");
    CTREX_HIP(c, nn::launch_conv3_head(in, in_cs, in_off, wt, bias, act, act_cs, act_off, h, hb, x,
                                       out_scale, mask, out, D, H, W,
                                       static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_scratch_bytes(int32_t cin, int32_t cout, int64_t n_vox, size_t *bytes) {
    if (!bytes) return CTREX_EINVAL;
    if (cin < 1 || cout < 1 || cin > 64 || cout > 64 || n_vox < 1) return CTREX_ESHAPE;
    size_t need = std::max(nn::conv3_wgrad_scratch(cin, cout, n_vox),
                           nn::upconv2_wgrad_scratch(cin, cout, n_vox));
    need = std::max(need, nn::channel_sum_scratch(cout));
    need = std::max(need, nn::head_bwd_scratch(16));
    need = std::max(need, sizeof(double) * (kMseBlocks + 1));
    *bytes = need;
    return CTREX_OK;
}

int ctrex_nn_conv3_wgrad(ctrex_ctx *c, const void *in, int32_t in_cs, int32_t in_off, int32_t cin,
                         const void *dout, int32_t dout_cs, int32_t dout_off, int32_t cout,
                         int32_t D, int32_t H, int32_t W, float *dw, float *dbias, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!(cin == 1 || chan_ok(cin)) || !chan_ok(cout) || (cin == 1 && cout != 16))
        return fail(c, CTREX_ESHAPE, "unsupported channels %d -> %d", cin, cout);
    if ((st = check_vol(c, D, H, W, false))) return st;
    if ((st = check_slice(c, "in", in, in_cs, in_off, cin, cin > 1))) return st;
    if ((st = check_slice(c, "dout", dout, dout_cs, dout_off, cout, true))) return st;
    if (!dw) return fail(c, CTREX_EINVAL, "dw is NULL");
    const long long n = static_cast<long long>(D) * H * W;
    const size_t need = std::max(nn::conv3_wgrad_scratch(cin, cout, n), nn::channel_sum_scratch(cout));
    void *scr;
    if ((st = ctx_scratch(c, need, &scr))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the tiled weight gradient sums the bias gradient as it stages dout
    CTREX_HIP(c, nn::launch_conv3_wgrad(in, in_cs, in_off, cin, nullptr, 0, 0, 0, dout, dout_cs,
                                        dout_off, cout, D, H, W, dw, cin > 1 ? dbias : nullptr,
                                        static_cast<float *>(scr), s));
    if (dbias && cin == 1)
        CTREX_HIP(c, nn::launch_channel_sum(dout, dout_cs, dout_off, cout, n, dbias,
                                            static_cast<double *>(scr), s));
    return CTREX_OK;
}

int ctrex_nn_conv3_wgrad_cat(ctrex_ctx *c, const void *in_a, int32_t a_cs, int32_t a_off,
                             int32_t ca, const void *in_b, int32_t b_cs, int32_t b_off, int32_t cb,
                             const void *dout, int32_t dout_cs, int32_t dout_off, int32_t cout,
                             int32_t D, int32_t H, int32_t W, float *dw, float *dbias,
                             void *stream) {
    int st = begin(c);
    if (st) return st;
    const int cin = ca + cb;
    if (!chan_ok(ca) || !(cb == 0 || chan_ok(cb)) || cin > 64 || !chan_ok(cout))
        return fail(c, CTREX_ESHAPE, "unsupported channels %d + %d -> %d", ca, cb, cout);
    if ((st = check_vol(c, D, H, W, false))) return st;
    if ((st = check_slice(c, "in_a", in_a, a_cs, a_off, ca, true))) return st;
    if (cb > 0 && (st = check_slice(c, "in_b", in_b, b_cs, b_off, cb, true))) return st;
    if ((st = check_slice(c, "dout", dout, dout_cs, dout_off, cout, true))) return st;
    if (!dw) return fail(c, CTREX_EINVAL, "dw is NULL");
    const long long n = static_cast<long long>(D) * H * W;
    const size_t need = std::max(nn::conv3_wgrad_scratch(cin, cout, n), nn::channel_sum_scratch(cout));
    void *scr;
    if ((st = ctx_scratch(c, need, &scr))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    CTREX_HIP(c, nn::launch_conv3_wgrad(in_a, a_cs, a_off, ca, in_b, b_cs, b_off, cb, dout, dout_cs,
                                        dout_off, cout, D, H, W, dw, dbias,
                                        static_cast<float *>(scr), s));
    return CTREX_OK;
}

int ctrex_nn_upconv2(ctrex_ctx *c, const void *in, int32_t in_cs, int32_t in_off, int32_t cin,
                     const void *wt, const float *bias, void *out, int32_t out_cs, int32_t out_off,
                     int32_t cout, int32_t D, int32_t H, int32_t W, uint32_t flags, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!((cin == 64 && cout == 32) || (cin == 32 && cout == 16) || (cin == 32 && cout == 32) ||
          (cin == 64 && cout == 64)))
        return fail(c, CTREX_ESHAPE, "unsupported channels %d -> %d", cin, cout);
    if (flags & ~(CTREX_NN_ACCUMULATE | CTREX_NN_OUT_F32)) return fail(c, CTREX_EINVAL, "bad flags");
    if ((st = check_vol(c, D, H, W, false))) return st;
    if ((st = check_slice(c, "in", in, in_cs, in_off, cin, true))) return st;
    if ((st = check_slice(c, "out", out, out_cs, out_off, cout, false))) return st;
    if (!wt) return fail(c, CTREX_EINVAL, "wt is NULL");
    CTREX_HIP(c, nn::launch_upconv2(in, in_cs, in_off, cin, wt, bias, out, out_cs, out_off, cout, D,
                                    H, W, flags & CTREX_NN_ACCUMULATE, flags & CTREX_NN_OUT_F32,
                                    static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_upconv2_dgrad(ctrex_ctx *c, const void *dout, int32_t dout_cs, int32_t dout_off,
                           int32_t cout, const void *wt_d, void *din, int32_t din_cs,
                           int32_t din_off, int32_t cin, int32_t D, int32_t H, int32_t W,
                           uint32_t flags, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!((cin == 64 && cout == 32) || (cin == 32 && cout == 16) || (cin == 32 && cout == 32) ||
          (cin == 64 && cout == 64)))
        return fail(c, CTREX_ESHAPE, "unsupported channels %d -> %d", cin, cout);
    if (flags & ~CTREX_NN_ACCUMULATE) return fail(c, CTREX_EINVAL, "bad flags");
    if ((st = check_vol(c, D, H, W, false))) return st;
    if ((st = check_slice(c, "dout", dout, dout_cs, dout_off, cout, true))) return st;
    if ((st = check_slice(c, "din", din, din_cs, din_off, cin, false))) return st;
    if (!wt_d) return fail(c, CTREX_EINVAL, "wt_d is NULL");
    CTREX_HIP(c, nn::launch_upconv2_dgrad(dout, dout_cs, dout_off, cout, wt_d, din, din_cs, din_off,
                                          cin, D, H, W, flags & CTREX_NN_ACCUMULATE,
                                          static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_upconv2_wgrad(ctrex_ctx *c, const void *in, int32_t in_cs, int32_t in_off,
                           int32_t cin, const void *dout, int32_t dout_cs, int32_t dout_off,
                           int32_t cout, int32_t D, int32_t H, int32_t W, float *dw, float *dbias,
                           void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!((cin == 64 && cout == 32) || (cin == 32 && cout == 16) || (cin == 32 && cout == 32) ||
          (cin == 64 && cout == 64)))
        return fail(c, CTREX_ESHAPE, "unsupported channels %d -> %d", cin, cout);
    if ((st = check_vol(c, D, H, W, false))) return st;
    if ((st = check_slice(c, "in", in, in_cs, in_off, cin, false))) return st;
    if ((st = check_slice(c, "dout", dout, dout_cs, dout_off, cout, true))) return st;
    if (!dw) return fail(c, CTREX_EINVAL, "dw is NULL");
    const long long n = static_cast<long long>(D) * H * W;
    const size_t need = std::max(nn::upconv2_wgrad_scratch(cin, cout, n), nn::channel_sum_scratch(cout));
    void *scr;
    if ((st = ctx_scratch(c, need, &scr))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    CTREX_HIP(c, nn::launch_upconv2_wgrad(in, in_cs, in_off, cin, dout, dout_cs, dout_off, cout, D,
                                          H, W, dw, static_cast<float *>(scr), s));
    if (dbias)
        CTREX_HIP(c, nn::launch_channel_sum(dout, dout_cs, dout_off, cout, 8 * n, dbias,
                                            static_cast<double *>(scr), s));
    return CTREX_OK;
}

int ctrex_nn_maxpool2(ctrex_ctx *c, const void *in, int32_t in_cs, int32_t in_off, int32_t ch,
                      void *out, int32_t D, int32_t H, int32_t W, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (ch < 1) return fail(c, CTREX_ESHAPE, "c must be >= 1");
    if (D < 2 || H < 2 || W < 2 || D % 2 || H % 2 || W % 2)
        return fail(c, CTREX_ESHAPE, "pooling needs even sides >= 2");
    if ((st = check_slice(c, "in", in, in_cs, in_off, ch, false))) return st;
    if (!out) return fail(c, CTREX_EINVAL, "out is NULL");
    CTREX_HIP(c, nn::launch_maxpool2(in, in_cs, in_off, ch, out, D, H, W, static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_maxpool2_backward(ctrex_ctx *c, const void *in, int32_t in_cs, int32_t in_off,
                               int32_t ch, const void *dout, void *din, int32_t D, int32_t H,
                               int32_t W, void *stream) {
    return maxpool2_backward(c, in, in_cs, in_off, ch, dout, din, D, H, W, false, stream);
}

int ctrex_nn_maxpool2_relu_backward(ctrex_ctx *c, const void *in, int32_t in_cs, int32_t in_off,
                                    int32_t ch, const void *dout, void *din, int32_t D, int32_t H,
                                    int32_t W, void *stream) {
    return maxpool2_backward(c, in, in_cs, in_off, ch, dout, din, D, H, W, true, stream);
}

int ctrex_nn_relu_backward(ctrex_ctx *c, const void *y, void *g, int32_t cs, int32_t off,
                           int32_t ch, int64_t n_vox, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (n_vox < 0 || ch < 1) return fail(c, CTREX_ESHAPE, "bad sizes");
    if ((st = check_slice(c, "y", y, cs, off, ch, false))) return st;
    if (!g) return fail(c, CTREX_EINVAL, "g is NULL");
    if (n_vox == 0) return CTREX_OK;
    CTREX_HIP(c, nn::launch_relu_bwd(y, g, cs, off, ch, n_vox, static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_input(ctrex_ctx *c, const float *x, float scale, void *xb, int64_t n_vox,
                   void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!x || !xb) return fail(c, CTREX_EINVAL, "NULL pointer");
    if (n_vox < 0) return fail(c, CTREX_ESHAPE, "bad sizes");
    if (!std::isfinite(scale) || scale == 0.0f) return fail(c, CTREX_EINVAL, "scale must be finite and non-zero");
    if (n_vox == 0) return CTREX_OK;
    CTREX_HIP(c, nn::launch_scale_bf16(x, scale, xb, n_vox, static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_head(ctrex_ctx *c, const void *act, int32_t ch, const float *h, const float *b,
                  const float *x, float out_scale, const float *mask, float *out, int64_t n_vox,
                  void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!act || !h || !b || !x || !out) return fail(c, CTREX_EINVAL, "NULL pointer");
    if (ch < 1 || ch > 64 || n_vox < 0) return fail(c, CTREX_ESHAPE, "bad sizes");
    if (!std::isfinite(out_scale)) return fail(c, CTREX_EINVAL, "out_scale must be finite");
    if (n_vox == 0) return CTREX_OK;
    CTREX_HIP(c, nn::launch_head(act, ch, h, b, x, out_scale, mask, out, n_vox,
                                 static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_head_backward(ctrex_ctx *c, const void *act, int32_t ch, const float *h,
                           float out_scale, const float *mask, const float *dout, void *dact,
                           float *dh, float *db, int64_t n_vox, void *stream) {
    return head_backward(c, act, ch, h, out_scale, mask, dout, dact, dh, db, n_vox, false, stream);
}

int ctrex_nn_head_relu_backward(ctrex_ctx *c, const void *act, int32_t ch, const float *h,
                                float out_scale, const float *mask, const float *dout, void *dact,
                                float *dh, float *db, int64_t n_vox, void *stream) {
    return head_backward(c, act, ch, h, out_scale, mask, dout, dact, dh, db, n_vox, true, stream);
}

int ctrex_nn_mse(ctrex_ctx *c, const float *a, const float *t, int64_t n, float weight,
                 double *loss, float *grad, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!a || !t) return fail(c, CTREX_EINVAL, "NULL pointer");
    if (n < 1) return fail(c, CTREX_ESHAPE, "n must be >= 1");
    if (!std::isfinite(weight)) return fail(c, CTREX_EINVAL, "weight must be finite");
    const int blocks = kMseBlocks;
    void *scr;
    if ((st = ctx_scratch(c, sizeof(double) * (blocks + 1), &scr))) return st;
    double *part = static_cast<double *>(scr);
    hipStream_t s = static_cast<hipStream_t>(stream);
    CTREX_HIP(c, nn::launch_mse(a, t, n, weight, grad, part, blocks, s));
    if (loss) {
        CTREX_HIP(c, launch_sum_partials(part, blocks, part + blocks, s));
        double h = 0.0;
        CTREX_HIP(c, hipMemcpyAsync(&h, part + blocks, sizeof h, hipMemcpyDeviceToHost, s));
        CTREX_HIP(c, hipStreamSynchronize(s));
        *loss = static_cast<double>(weight) * h / static_cast<double>(n);
    }
    return CTREX_OK;
}

int ctrex_nn_adam(ctrex_ctx *c, float *param, const float *grad, float *m, float *v, int64_t n,
                  float lr, float beta1, float beta2, float eps, int32_t step, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!param || !grad || !m || !v) return fail(c, CTREX_EINVAL, "NULL pointer");
    if (n < 0 || step < 1) return fail(c, CTREX_EINVAL, "n >= 0 and step >= 1 required");
    if (n == 0) return CTREX_OK;
    CTREX_HIP(c, nn::launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, step,
                                 static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_pack_conv3(ctrex_ctx *c, const float *w, int32_t cout, int32_t cin, void *wt,
                        void *wt_d, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!w) return fail(c, CTREX_EINVAL, "w is NULL");
    if (cout < 1 || cin < 1) return fail(c, CTREX_ESHAPE, "bad channel counts");
    CTREX_HIP(c, nn::launch_pack(w, cout, cin, 27, true, wt, wt_d, false,
                                 static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

int ctrex_nn_pack_upconv2(ctrex_ctx *c, const float *w, int32_t cin, int32_t cout, void *wt,
                          void *wt_d, void *stream) {
    int st = begin(c);
    if (st) return st;
    if (!w) return fail(c, CTREX_EINVAL, "w is NULL");
    if (cout < 1 || cin < 1) return fail(c, CTREX_ESHAPE, "bad channel counts");
    CTREX_HIP(c, nn::launch_pack(w, cout, cin, 8, false, wt, wt_d, true,
                                 static_cast<hipStream_t>(stream)));
    return CTREX_OK;
}

}  // extern "C"
