// Native executor of the learned warm start (a 3-level 3D U-Net): parameter
// layout, workspace planning, forward, backward, Adam, and the C ABI entry
// points ws_* declared in pmeft.h.
#include "pmeft_internal.h"

#include <math.h>
#include <string.h>

namespace pmeft {

// kernels (unet_kernels.hip)
void launch_conv3(const uint16_t *in, int in_stride, int in_off, int cin_pad, const uint16_t *wp, int cout_pad,
                  const float *bias, int cout, void *out, int out_stride, int out_off, bool out_f32, int n, bool flip,
                  bool relu, hipStream_t st);
void launch_conv3_wgrad(const uint16_t *x, int x_stride, int x_off, int cin, const uint16_t *dy, int dy_stride,
                        int dy_off, int cout, float *dw, float *db, float *part, int n, hipStream_t st);
size_t wgrad_partial_floats(int cin, int cout);
void launch_relu_bwd(uint16_t *dy, int dstride, int doff, const uint16_t *y, int ystride, int yoff, int C,
                     unsigned nvox, hipStream_t st);
void launch_pool(const uint16_t *in, int istride, int ioff, uint16_t *out, int ostride, int ooff, int C, int nc,
                 hipStream_t st);
void launch_pool_bwd(const uint16_t *dout, int ostride, int ooff, uint16_t *din, int istride, int ioff, int C, int nf,
                     hipStream_t st);
void launch_up(const uint16_t *in, int istride, int ioff, uint16_t *out, int ostride, int ooff, int C, int nf,
               hipStream_t st);
void launch_up_bwd(const uint16_t *dout, int ostride, int ooff, uint16_t *din, int istride, int ioff, int C, int nc,
                   hipStream_t st);
void launch_feature_stats(const double *delta_packed, unsigned long long n3, ReduceSlot rs, hipStream_t st);
void launch_unet_input(const double *delta_packed, int n, const double *stats, float ab0, float am0, float a,
                       uint16_t *x0, hipStream_t st);
void launch_source_target(const double *chi, const double *delta_packed, int n, double inv_scale, float *t,
                          hipStream_t st);
void launch_add_source(const float *yhat, int n, double *delta_packed, ReduceSlot rs, hipStream_t st);
void launch_head(const uint16_t *b5, const float *hw, const float *hb, unsigned nvox, float *yhat, hipStream_t st);
void launch_head_loss_bwd(const float *yhat, const float *y, const uint16_t *b5, const float *hw, unsigned nvox,
                          uint16_t *db5, float *ghw, float *ghb, float *loss, float *part, hipStream_t st);
size_t head_partial_floats();
void launch_bf16_slice_to_f32(const uint16_t *s, int stride, int off, int C, float *d, size_t nvox, hipStream_t st);
void launch_pack_conv(const float *w, int cin, int cout, int cin_pad, int cout_pad, uint16_t *wf, uint16_t *wd,
                      hipStream_t st);
void launch_adam(float *w, const float *g, float *m, float *v, long long n, double lr, double b1, double b2,
                 double eps, long long step, const double *gsq, double clip, hipStream_t st);
void launch_sumsq(const float *g, long long n, ReduceSlot rs, hipStream_t st);
void launch_f32_to_bf16(const float *s, uint16_t *d, size_t n, hipStream_t st);
void launch_pack_poly(const float *w, int cin, int cout, int cup, int cout_pad, uint16_t *wp, hipStream_t st);
void launch_pack_conv_sub(const float *w, int cin, int cout, int c0, int csub, int csub_pad, int cout_pad,
                          uint16_t *wf, hipStream_t st);
bool launch_upconv_poly(const uint16_t *in, int cup, int nc, const uint16_t *wp, int cout_pad, const float *bias,
                        const float *add, int cout, void *out, int out_stride, int out_off, bool out_f32, bool relu,
                        hipStream_t st);
bool launch_updec16(const uint16_t *skip, int skip_stride, int skip_off, const uint16_t *coarse, const uint16_t *wsub,
                    const uint16_t *wpoly, const float *bias, void *out, int out_stride, int out_off, bool out_f32,
                    bool relu, int n, hipStream_t st);
void launch_unet_feature(const double *delta_packed, int n, const double *stats, uint16_t *f, hipStream_t st);
bool launch_conv3_in1(const uint16_t *f, const float *w, const float *b, float x1, float x2, float x3, void *out,
                      int out_stride, int out_off, bool out_f32, int n, hipStream_t st);
bool launch_conv3_head(const uint16_t *in, int in_stride, int in_off, const uint16_t *wp, const float *bias,
                       const float *hw, const float *hb, float *yhat, int n, hipStream_t st);
namespace {

struct ConvSpec {
    int cin, cout;
};
// l1a l1b l2a l2b l3a l3b l4a l4b l5a l5b
constexpr ConvSpec kConv[10] = {{4, 16},  {16, 16}, {16, 32}, {32, 32}, {32, 64},
                                {64, 64}, {96, 32}, {32, 32}, {48, 16}, {16, 16}};

inline int pad16(int c) { return (c + 15) / 16 * 16; }

struct ParamLayout {
    long long w[10], b[10], hw, hb, total;
};

ParamLayout param_layout()
{
    ParamLayout L;
    long long o = 0;
    for (int l = 0; l < 10; l++) {
        L.w[l] = o;
        o += 27LL * kConv[l].cin * kConv[l].cout;
        L.b[l] = o;
        o += kConv[l].cout;
    }
    L.hw = o;
    o += 16;
    L.hb = o;
    o += 1;
    L.total = o;
    return L;
}

// activation tensors: name, level (0: n, 1: n/2, 2: n/4), channels
enum { X0, A1, C1, P1, A2, C2, P2, A3, B3, A4, B4, A5, B5, NT };
constexpr int kTLevel[NT] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 1, 1, 0, 0};
constexpr int kTChan[NT] = {16, 16, 48, 16, 32, 96, 32, 64, 64, 32, 32, 16, 16};

// The decoder layers whose input is [upsampled | skip] (l4a: 64 | 32 channels,
// l5a: 32 | 16): at inference they run as a convolution of the skip channels
// (FP32 result) plus the polyphase convolution of the coarse tensor, with no
// upsampled tensor in memory.
constexpr int kFused[2] = {6, 8};
constexpr int kFusedUp[2] = {64, 32};

struct NetPlan {
    int n = 0;
    bool training = false;
    size_t total = 0;
    size_t red_partials = 0, red_out = 0;
    size_t wf[10] = {}, wd[10] = {};
    size_t wpoly[2] = {}, wsub[2] = {};  // inference: polyphase and skip-channel weights of kFused
    size_t act[NT] = {}, grad[NT] = {};
    size_t delta = 0, yhat = 0, target = 0, pgrad = 0, loss = 0, wg_part = 0;
};

size_t take(size_t &cur, size_t bytes)
{
    const size_t o = cur;
    cur += (bytes + 255) & ~(size_t)255;
    return o;
}

bool net_plan(NetPlan &P, int n, bool training)
{
    if (n < 64 || n > 1024 || n % 64)
        return false;
    P = NetPlan();
    P.n = n;
    P.training = training;
    size_t c = 0;
    P.red_partials = take(c, sizeof(double) * 8 * kMaxBlocks);
    P.red_out = take(c, sizeof(double) * 8);
    for (int l = 0; l < 10; l++) {
        const size_t sz = sizeof(uint16_t) * 27 * pad16(kConv[l].cin) * pad16(kConv[l].cout);
        P.wf[l] = take(c, sz);
        if (training && l > 0)
            P.wd[l] = take(c, sz);
    }
    if (!training)
        for (int f = 0; f < 2; f++) {
            const int l = kFused[f], cout_pad = pad16(kConv[l].cout);
            P.wpoly[f] = take(c, sizeof(uint16_t) * 64 * cout_pad * kFusedUp[f]);
            P.wsub[f] = take(c, sizeof(uint16_t) * 27 * cout_pad * pad16(kConv[l].cin - kFusedUp[f]));
        }
    for (int t = 0; t < NT; t++) {
        const size_t m = (size_t)(n >> kTLevel[t]);
        const size_t sz = sizeof(uint16_t) * m * m * m * kTChan[t];
        P.act[t] = take(c, sz);
        if (training && t != X0)
            P.grad[t] = take(c, sz);
    }
    const size_t n3 = (size_t)n * n * n;
    P.delta = take(c, sizeof(double) * n3);
    P.yhat = take(c, sizeof(float) * n3);
    if (training) {
        P.target = take(c, sizeof(float) * n3);
        P.pgrad = take(c, sizeof(float) * param_layout().total);
        P.loss = take(c, 256);
        size_t wmax = head_partial_floats();
        for (int l = 0; l < 10; l++) {
            const size_t f = wgrad_partial_floats(kConv[l].cin, kConv[l].cout);
            wmax = wmax > f ? wmax : f;
        }
        P.wg_part = take(c, sizeof(float) * wmax);
    }
    P.total = c + 256;
    return true;
}

struct Net {
    NetPlan P;
    char *ws;
    hipStream_t st;
    ReduceSlot rs;
    uint16_t *act(int t) const { return (uint16_t *)(ws + P.act[t]); }
    uint16_t *grad(int t) const { return (uint16_t *)(ws + P.grad[t]); }
    int dim(int t) const { return P.n >> kTLevel[t]; }
    unsigned nvox(int t) const { return (unsigned)dim(t) * dim(t) * dim(t); }
};

int launched() { return hipGetLastError() == hipSuccess ? PM_OK : PM_EHIP; }

// every weight layout the network's kernels read, in one launch
void pack_all(Net &N, const float *params)
{
    const ParamLayout L = param_layout();
    PackJobs J{};
    for (int l = 0; l < 10; l++)
        J.job[J.n++] = PackJob{0, params + L.w[l], kConv[l].cin, kConv[l].cout, pad16(kConv[l].cin),
                               pad16(kConv[l].cout), 0, 0, (uint16_t *)(N.ws + N.P.wf[l]),
                               N.P.wd[l] ? (uint16_t *)(N.ws + N.P.wd[l]) : nullptr};
    if (!N.P.training)
        for (int f = 0; f < 2; f++) {
            const int l = kFused[f], cin = kConv[l].cin, cout = kConv[l].cout, up = kFusedUp[f];
            J.job[J.n++] = PackJob{1, params + L.w[l], cin, cout, up, pad16(cout), 0, 0,
                                   (uint16_t *)(N.ws + N.P.wpoly[f]), nullptr};
            J.job[J.n++] = PackJob{2, params + L.w[l], cin, cout, up, cin - up, pad16(cin - up), pad16(cout),
                                   (uint16_t *)(N.ws + N.P.wsub[f]), nullptr};
        }
    launch_pack_jobs(J, N.st);
}

// A slice of an activation tensor: tensor t, voxel stride, channel offset.
struct View {
    int t, stride, off;
};
View whole(int t) { return View{t, kTChan[t], 0}; }

// Inference form of decoder layer kFused[f] (skip channels in view `skip`,
// coarse tensor tc, output to): the skip channels' convolution into an FP32
// scratch (the input and first activation tensors, dead by then), then the
// polyphase convolution of tc adds it, the bias and the ReLU; the layer on
// the 16-channel level runs both in one kernel (the same values).
// Needs N.dim(tc) % 64 == 0 (the polyphase instances).
void fused_up_conv(Net &N, const float *params, int f, View skip, int tc, int to)
{
    const ParamLayout L = param_layout();
    const int l = kFused[f], cin = kConv[l].cin, cout = kConv[l].cout, up = kFusedUp[f];
    if (cin - up == 16 && up == 32 && cout == 16 &&
        launch_updec16(N.act(skip.t), skip.stride, skip.off, N.act(tc), (const uint16_t *)(N.ws + N.P.wsub[f]),
                       (const uint16_t *)(N.ws + N.P.wpoly[f]), params + L.b[l], N.act(to), kTChan[to], 0, false,
                       true, N.dim(to), N.st))
        return;
    float *scratch = (float *)N.act(X0);
    launch_conv3(N.act(skip.t), skip.stride, skip.off, pad16(cin - up), (const uint16_t *)(N.ws + N.P.wsub[f]),
                 pad16(cout), nullptr, cout, scratch, cout, 0, true, N.dim(to), false, false, N.st);
    launch_upconv_poly(N.act(tc), up, N.dim(tc), (const uint16_t *)(N.ws + N.P.wpoly[f]), pad16(cout),
                       params + L.b[l], scratch, cout, N.act(to), kTChan[to], 0, false, true, N.st);
}

// conv layer l (ReLU) from view vi into view vo
void conv_fwd(Net &N, const float *params, int l, View vi, View vo)
{
    const ParamLayout L = param_layout();
    launch_conv3(N.act(vi.t), vi.stride, vi.off, pad16(kConv[l].cin), (const uint16_t *)(N.ws + N.P.wf[l]),
                 pad16(kConv[l].cout), params + L.b[l], kConv[l].cout, N.act(vo.t), vo.stride, vo.off, false,
                 N.dim(vo.t), false, true, N.st);
}

// delta: packed, mean-free density contrast.  Training keeps every
// activation the backward pass reads, in the concatenation layout.
// Inference (all exact rewrites of the same network): the first layer runs
// on the density channel alone with the broadcast channels folded into its
// bias; the two decoder layers that read upsampled tensors run in the
// polyphase form (no upsampled tensor; their skip tensors then live in
// compact views, not in the concatenation buffers); the last layer applies
// the output head in its epilogue.
void forward(Net &N, const float *params, const double *delta, const pm_eft_params &p)
{
    const int n = N.P.n;
    const unsigned nv = (unsigned)n * n * n;
    const ParamLayout L = param_layout();
    const bool infer = !N.P.training;
    const bool poly0 = infer && N.dim(B3) % 64 == 0, poly1 = infer && N.dim(B4) % 64 == 0;
    const View s1 = poly1 ? View{C1, 16, 0} : View{C1, 48, 32};  // skip 1
    const View s2 = poly0 ? View{C2, 32, 0} : View{C2, 96, 64};  // skip 2
    launch_feature_stats(delta, nv, N.rs, N.st);
    bool first = false;
    if (infer) {
        launch_unet_feature(delta, n, N.rs.out, N.act(X0), N.st);
        first = launch_conv3_in1(N.act(X0), params + L.w[0], params + L.b[0], (float)p.alpha_b0, (float)p.alpha_m0,
                                 (float)p.a, N.act(A1), kTChan[A1], 0, false, n, N.st);
    }
    if (!first) {
        launch_unet_input(delta, n, N.rs.out, (float)p.alpha_b0, (float)p.alpha_m0, (float)p.a, N.act(X0), N.st);
        conv_fwd(N, params, 0, whole(X0), whole(A1));
    }
    conv_fwd(N, params, 1, whole(A1), s1);
    launch_pool(N.act(C1), s1.stride, s1.off, N.act(P1), 16, 0, 16, n / 2, N.st);
    conv_fwd(N, params, 2, whole(P1), whole(A2));
    conv_fwd(N, params, 3, whole(A2), s2);
    launch_pool(N.act(C2), s2.stride, s2.off, N.act(P2), 32, 0, 32, n / 4, N.st);
    conv_fwd(N, params, 4, whole(P2), whole(A3));
    conv_fwd(N, params, 5, whole(A3), whole(B3));
    if (poly0) {
        fused_up_conv(N, params, 0, s2, B3, A4);
    } else {
        launch_up(N.act(B3), 64, 0, N.act(C2), 96, 0, 64, n / 2, N.st);
        conv_fwd(N, params, 6, whole(C2), whole(A4));
    }
    conv_fwd(N, params, 7, whole(A4), whole(B4));
    if (poly1) {
        fused_up_conv(N, params, 1, s1, B4, A5);
    } else {
        launch_up(N.act(B4), 32, 0, N.act(C1), 48, 0, 32, n, N.st);
        conv_fwd(N, params, 8, whole(C1), whole(A5));
    }
    float *yhat = (float *)(N.ws + N.P.yhat);
    if (infer && launch_conv3_head(N.act(A5), kTChan[A5], 0, (const uint16_t *)(N.ws + N.P.wf[9]), params + L.b[9],
                                   params + L.hw, params + L.hb, yhat, n, N.st))
        return;
    conv_fwd(N, params, 9, whole(A5), whole(B5));
    launch_head(N.act(B5), params + L.hw, params + L.hb, nv, yhat, N.st);
}

// backward of conv layer l given the (already ReLU-masked) output gradient
// (tg, goff): weight and bias gradients, and the input gradient into
// (gi, gioff) unless gi < 0.
void conv_bwd(Net &N, int l, int ti, int ioff, int tg, int goff, int gi, int gioff)
{
    const ParamLayout L = param_layout();
    float *pg = (float *)(N.ws + N.P.pgrad);
    launch_conv3_wgrad(N.act(ti), kTChan[ti], ioff, kConv[l].cin, N.grad(tg), kTChan[tg], goff, kConv[l].cout,
                       pg + L.w[l], pg + L.b[l], (float *)(N.ws + N.P.wg_part), N.dim(tg), N.st);
    if (gi >= 0)
        launch_conv3(N.grad(tg), kTChan[tg], goff, pad16(kConv[l].cout), (const uint16_t *)(N.ws + N.P.wd[l]),
                     pad16(kConv[l].cin), nullptr, kConv[l].cin, N.grad(gi), kTChan[gi], gioff, false, N.dim(gi),
                     true, false, N.st);
}

void mask(Net &N, int tg, int goff, int ta, int aoff, int C)
{
    launch_relu_bwd(N.grad(tg), kTChan[tg], goff, N.act(ta), kTChan[ta], aoff, C, N.nvox(ta), N.st);
}

// Gradients of every parameter into the workspace's pgrad.  dy: dL/dyhat
// (ng^3 FP32, natural order); null: the MSE loss against the workspace's
// target t, whose mean goes to the workspace's loss slot.  Every gradient is
// written, not accumulated, in a fixed order.
void backward(Net &N, const float *params, const float *dy)
{
    const int n = N.P.n;
    const unsigned nv = (unsigned)n * n * n;
    const ParamLayout L = param_layout();
    float *pg = (float *)(N.ws + N.P.pgrad);
    if (dy)
        launch_head_loss_bwd(dy, nullptr, N.act(B5), params + L.hw, nv, N.grad(B5), pg + L.hw, pg + L.hb, nullptr,
                             (float *)(N.ws + N.P.wg_part), N.st);
    else
        launch_head_loss_bwd((const float *)(N.ws + N.P.yhat), (const float *)(N.ws + N.P.target), N.act(B5),
                             params + L.hw, nv, N.grad(B5), pg + L.hw, pg + L.hb, (float *)(N.ws + N.P.loss),
                             (float *)(N.ws + N.P.wg_part), N.st);
    conv_bwd(N, 9, A5, 0, B5, 0, A5, 0);
    mask(N, A5, 0, A5, 0, 16);
    conv_bwd(N, 8, C1, 0, A5, 0, C1, 0);
    launch_up_bwd(N.grad(C1), 48, 0, N.grad(B4), 32, 0, 32, n / 2, N.st);
    mask(N, B4, 0, B4, 0, 32);
    conv_bwd(N, 7, A4, 0, B4, 0, A4, 0);
    mask(N, A4, 0, A4, 0, 32);
    conv_bwd(N, 6, C2, 0, A4, 0, C2, 0);
    launch_up_bwd(N.grad(C2), 96, 0, N.grad(B3), 64, 0, 64, n / 4, N.st);
    mask(N, B3, 0, B3, 0, 64);
    conv_bwd(N, 5, A3, 0, B3, 0, A3, 0);
    mask(N, A3, 0, A3, 0, 64);
    conv_bwd(N, 4, P2, 0, A3, 0, P2, 0);
    launch_pool_bwd(N.grad(P2), 32, 0, N.grad(C2), 96, 64, 32, n / 2, N.st);  // + skip 2
    mask(N, C2, 64, C2, 64, 32);
    conv_bwd(N, 3, A2, 0, C2, 64, A2, 0);
    mask(N, A2, 0, A2, 0, 32);
    conv_bwd(N, 2, P1, 0, A2, 0, P1, 0);
    launch_pool_bwd(N.grad(P1), 16, 0, N.grad(C1), 48, 32, 16, n, N.st);  // + skip 1
    mask(N, C1, 32, C1, 32, 16);
    conv_bwd(N, 1, A1, 0, C1, 32, A1, 0);
    mask(N, A1, 0, A1, 0, 16);
    conv_bwd(N, 0, X0, 0, A1, 0, -1, 0);
}

int setup(Net &N, int n, bool training, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    if (!ws || ((uintptr_t)ws & 255))
        return PM_EINVAL;
    if (!net_plan(N.P, n, training))
        return PM_EINVAL;
    if (ws_bytes < N.P.total)
        return PM_ENOMEM;
    N.ws = (char *)ws;
    N.st = (hipStream_t)stream;
    N.rs.partials = (double *)(N.ws + N.P.red_partials);
    N.rs.counter = nullptr;
    N.rs.out = (double *)(N.ws + N.P.red_out);
    return PM_OK;
}

double source_scale(int n, const pm_eft_params &p)
{
    pm_eft_coeffs c;
    pm_eft_coefficients(&p, &c);
    const double h = 1.0 / n;
    return h * h * c.s * c.mu_chi;
}

// natural rho -> packed mean-free delta in the workspace
double *prepare_input(Net &N, const double *rho)
{
    const int n = N.P.n;
    const long long n3 = (long long)n * n * n;
    double *d = (double *)(N.ws + N.P.delta);
    launch_natural_to_packed(rho, PM_F64, d, n, 1.0, 0.0, N.st);
    launch_field_sum(d, n3, N.rs, N.st);
    launch_subtract_mean(d, n3, N.rs.out, N.st);
    return d;
}

}  // namespace
}  // namespace pmeft

namespace pmeft {

// The learned source for the solver, in two parts: the forward pass (the
// packed delta saved into `save`, ng^3 doubles, and the network run on that
// copy), then delta <- delta + t - <t>.
int unet_learned_forward(const float *params, const double *delta_packed, double *save, int ng,
                         const pm_eft_params &p, void *ws, size_t ws_bytes, hipStream_t st, bool packed)
{
    Net N;
    int e = setup(N, ng, false, ws, ws_bytes, st);
    if (e)
        return e;
    const size_t n3 = (size_t)ng * ng * ng;
    if (hipMemcpyAsync(save, delta_packed, sizeof(double) * n3, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return PM_EHIP;
    if (!packed)
        pack_all(N, params);
    forward(N, params, save, p);
    return launched();
}

int unet_learned_pack(const float *params, int ng, void *ws, size_t ws_bytes, hipStream_t st)
{
    Net N;
    int e = setup(N, ng, false, ws, ws_bytes, st);
    if (e)
        return e;
    pack_all(N, params);
    return launched();
}

int unet_add_learned_source(void *ws, int ng, double *delta_packed, hipStream_t st)
{
    NetPlan P;
    if (!net_plan(P, ng, false))
        return PM_EINVAL;
    ReduceSlot rs;
    rs.partials = (double *)((char *)ws + P.red_partials);
    rs.counter = nullptr;
    rs.out = (double *)((char *)ws + P.red_out);
    launch_add_source((const float *)((char *)ws + P.yhat), ng, delta_packed, rs, st);
    return launched();
}

// the learned-source workspace's save area (ng^3 doubles)
double *unet_save_area(void *ws, int ng)
{
    NetPlan P;
    if (!net_plan(P, ng, false))
        return nullptr;
    return (double *)((char *)ws + P.delta);
}

}  // namespace pmeft

using namespace pmeft;

extern "C" {

long long ws_unet_param_count(void) { return param_layout().total; }

size_t ws_unet_workspace_bytes(int ng, int training)
{
    NetPlan P;
    return net_plan(P, ng, training != 0) ? P.total : 0;
}

int ws_unet_forward(const float *params, const double *rho, int ng, const pm_eft_params *p, float *yhat_out,
                    void *ws, size_t ws_bytes, pm_stream_t stream)
{
    if (!params || !rho || !p || !yhat_out)
        return PM_EINVAL;
    Net N;
    int e = setup(N, ng, false, ws, ws_bytes, stream);
    if (e)
        return e;
    const double *d = prepare_input(N, rho);
    pack_all(N, params);
    forward(N, params, d, *p);
    const unsigned nv = (unsigned)ng * ng * ng;
    if (hipMemcpyAsync(yhat_out, N.ws + N.P.yhat, sizeof(float) * nv, hipMemcpyDeviceToDevice, N.st) != hipSuccess)
        return PM_EHIP;
    return launched();
}

int ws_unet_forward_train(const float *params, const double *rho, int ng, const pm_eft_params *p, float *yhat_out,
                          void *ws, size_t ws_bytes, pm_stream_t stream)
{
    if (!params || !rho || !p)
        return PM_EINVAL;
    Net N;
    int e = setup(N, ng, true, ws, ws_bytes, stream);
    if (e)
        return e;
    const double *d = prepare_input(N, rho);
    pack_all(N, params);
    forward(N, params, d, *p);
    const unsigned nv = (unsigned)ng * ng * ng;
    if (yhat_out &&
        hipMemcpyAsync(yhat_out, N.ws + N.P.yhat, sizeof(float) * nv, hipMemcpyDeviceToDevice, N.st) != hipSuccess)
        return PM_EHIP;
    return launched();
}

int ws_unet_backward(const float *params, const float *dloss_dyhat, int ng, float *grad_out, void *ws,
                     size_t ws_bytes, pm_stream_t stream)
{
    if (!params || !dloss_dyhat || !grad_out)
        return PM_EINVAL;
    Net N;
    int e = setup(N, ng, true, ws, ws_bytes, stream);
    if (e)
        return e;
    backward(N, params, dloss_dyhat);
    const long long np = param_layout().total;
    if (hipMemcpyAsync(grad_out, N.ws + N.P.pgrad, sizeof(float) * np, hipMemcpyDeviceToDevice, N.st) != hipSuccess)
        return PM_EHIP;
    return launched();
}

size_t ws_adam_workspace_bytes(long long n)
{
    (void)n;
    return sizeof(double) * 8 * kMaxBlocks + 256 + 256;
}

namespace {
int adam_impl(float *params, const float *grads, float *m, float *v, long long n, long long step, double lr,
              double b1, double b2, double eps, double grad_clip, ReduceSlot rs, hipStream_t st)
{
    launch_sumsq(grads, n, rs, st);
    launch_adam(params, grads, m, v, n, lr, b1, b2, eps, step, rs.out, grad_clip, st);
    return launched();
}
}  // namespace

int ws_adam_step(float *params, const float *grads, float *m, float *v, long long n, long long step, double lr,
                 double beta1, double beta2, double eps, double grad_clip, double *grad_norm, void *ws,
                 size_t ws_bytes, pm_stream_t stream)
{
    if (!params || !grads || !m || !v || n <= 0 || n > (1LL << 31) - 1 || step < 1 || !(lr >= 0.0) ||
        !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0) || !(grad_clip >= 0.0) ||
        !ws || ((uintptr_t)ws & 255))
        return PM_EINVAL;
    if (ws_bytes < ws_adam_workspace_bytes(n))
        return PM_ENOMEM;
    ReduceSlot rs;
    rs.partials = (double *)ws;
    rs.counter = nullptr;
    rs.out = (double *)((char *)ws + sizeof(double) * 8 * kMaxBlocks);
    hipStream_t st = (hipStream_t)stream;
    int e = adam_impl(params, grads, m, v, n, step, lr, beta1, beta2, eps, grad_clip, rs, st);
    if (e)
        return e;
    if (grad_norm) {
        double g2 = 0.0;
        if (hipMemcpyAsync(&g2, rs.out, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return PM_EHIP;
        *grad_norm = sqrt(g2);
    }
    return PM_OK;
}

int ws_unet_train_step(float *params, float *adam_m, float *adam_v, long long step, double lr, double grad_clip,
                       const double *rho, const double *chi_target, int ng, const pm_eft_params *p, float *grad_out,
                       double *loss, double *grad_norm, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    if (!params || !rho || !chi_target || !p || (lr > 0.0 && (!adam_m || !adam_v || step < 1)) || !(grad_clip >= 0.0))
        return PM_EINVAL;
    Net N;
    int e = setup(N, ng, true, ws, ws_bytes, stream);
    if (e)
        return e;
    const double sc = source_scale(ng, *p);
    if (!(sc != 0.0) || !isfinite(sc))
        return PM_EINVAL;
    const double *d = prepare_input(N, rho);
    launch_source_target(chi_target, d, ng, 1.0 / sc, (float *)(N.ws + N.P.target), N.st);
    pack_all(N, params);
    forward(N, params, d, *p);
    backward(N, params, nullptr);
    const long long np = param_layout().total;
    const float *pg = (const float *)(N.ws + N.P.pgrad);
    if (grad_out && hipMemcpyAsync(grad_out, pg, sizeof(float) * np, hipMemcpyDeviceToDevice, N.st) != hipSuccess)
        return PM_EHIP;
    if (lr > 0.0) {
        e = adam_impl(params, pg, adam_m, adam_v, np, step, lr, 0.9, 0.999, 1e-8, grad_clip, N.rs, N.st);
        if (e)
            return e;
    } else {
        launch_sumsq(pg, np, N.rs, N.st);
    }
    if (loss || grad_norm) {
        float l = 0.f;
        double g2 = 0.0;
        if (hipMemcpyAsync(&l, N.ws + N.P.loss, sizeof(float), hipMemcpyDeviceToHost, N.st) != hipSuccess ||
            hipMemcpyAsync(&g2, N.rs.out, sizeof(double), hipMemcpyDeviceToHost, N.st) != hipSuccess ||
            hipStreamSynchronize(N.st) != hipSuccess)
            return PM_EHIP;
        if (loss)
            *loss = l;
        if (grad_norm)
            *grad_norm = sqrt(g2);
    }
    return launched();
}

int ws_unet_tensor(const void *ws, int ng, int tensor, int gradient, float *out, pm_stream_t stream)
{
    NetPlan P;
    if (!ws || !out || tensor < 0 || tensor >= NT || !net_plan(P, ng, true) || (gradient && tensor == X0))
        return PM_EINVAL;
    const size_t m = (size_t)(ng >> kTLevel[tensor]);
    launch_bf16_slice_to_f32((const uint16_t *)((const char *)ws + (gradient ? P.grad[tensor] : P.act[tensor])),
                             kTChan[tensor], 0, kTChan[tensor], out, m * m * m, (hipStream_t)stream);
    return launched();
}

int ws_conv3(int mode, int n, int cin, int cout, const void *x_bf16, const void *dy_bf16, const float *w,
             const float *b, float *out, void *ws, size_t ws_bytes, pm_stream_t stream)
{
    if (mode < 0 || mode > 4 || n < 16 || n % 16 || cin < 1 || cout < 1 || cin > 96 || cout > 96 || !w || !out || !ws ||
        ((uintptr_t)ws & 255))
        return PM_EINVAL;
    // mode 4, b: [cout biases | head weights (16) | head bias]
    if (mode == 4 && (!x_bf16 || !b || cin != 16 || cout != 16 || n % 64))
        return PM_EINVAL;
    const size_t wbytes = ((sizeof(uint16_t) * 27 * pad16(cin) * pad16(cout)) + 255) & ~(size_t)255;
    const size_t need = 2 * wbytes + sizeof(float) * wgrad_partial_floats(cin, cout);
    if (ws_bytes < need)
        return PM_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    uint16_t *wf = (uint16_t *)ws;
    uint16_t *wd = (uint16_t *)((char *)ws + wbytes);
    float *part = (float *)((char *)ws + 2 * wbytes);
    if (mode == 3) {
        // decoder layer of the upsampled form: x = coarse (n/2)^3 x (2 cin / 3)
        // channels (upsampled part), dy = n^3 x (cin / 3) skip channels
        const int up = 2 * cin / 3, sub = cin - up;
        if (!x_bf16 || !dy_bf16 || cin % 3 || up % 32 || sub % 16 || n % 128)
            return PM_EINVAL;
        const size_t pbytes = ((sizeof(uint16_t) * 64 * pad16(cout) * up) + 255) & ~(size_t)255;
        if (pbytes + sizeof(uint16_t) * 27 * pad16(cout) * sub > 2 * wbytes)
            return PM_ENOMEM;
        uint16_t *wpoly = (uint16_t *)ws, *wsub = (uint16_t *)((char *)ws + pbytes);
        launch_pack_poly(w, cin, cout, up, pad16(cout), wpoly, st);
        launch_pack_conv_sub(w, cin, cout, up, sub, sub, pad16(cout), wsub, st);
        if (up == 32 && sub == 16 && cout == 16) {
            // the 16-channel level's layer: one fused kernel
            if (!launch_updec16((const uint16_t *)dy_bf16, sub, 0, (const uint16_t *)x_bf16, wsub, wpoly, b, out,
                                cout, 0, true, false, n, st))
                return PM_EINVAL;
            return launched();
        }
        launch_conv3((const uint16_t *)dy_bf16, sub, 0, sub, wsub, pad16(cout), nullptr, cout, out, cout, 0, true, n,
                     false, false, st);
        if (!launch_upconv_poly((const uint16_t *)x_bf16, up, n / 2, wpoly, pad16(cout), b, out, cout, out, cout, 0,
                                true, false, st))
            return PM_EINVAL;
        return launched();
    }
    launch_pack_conv(w, cin, cout, pad16(cin), pad16(cout), wf, wd, st);
    if (mode == 4) {
        if (!launch_conv3_head((const uint16_t *)x_bf16, 16, 0, wf, b, b + 16, b + 32, out, n, st))
            return PM_EINVAL;
        return launched();
    }
    if (mode == 0) {
        if (!x_bf16 || cin % 16)
            return PM_EINVAL;
        launch_conv3((const uint16_t *)x_bf16, cin, 0, cin, wf, pad16(cout), b, cout, out, cout, 0, true, n, false,
                     false, st);
    } else if (mode == 1) {
        if (!dy_bf16 || cout % 16)
            return PM_EINVAL;
        launch_conv3((const uint16_t *)dy_bf16, cout, 0, cout, wd, pad16(cin), nullptr, cin, out, cin, 0, true, n,
                     true, false, st);
    } else {
        if (!x_bf16 || !dy_bf16)
            return PM_EINVAL;
        launch_conv3_wgrad((const uint16_t *)x_bf16, cin, 0, cin, (const uint16_t *)dy_bf16, cout, 0, cout, out,
                           nullptr, part, n, st);
    }
    return launched();
}

int ws_conv3_first(int n, const void *f_bf16, const float *w, const float *b, const float *xc, float *out,
                   pm_stream_t stream)
{
    if (n < 64 || n % 64 || !f_bf16 || !w || !b || !xc || !out)
        return PM_EINVAL;
    if (!launch_conv3_in1((const uint16_t *)f_bf16, w, b, xc[0], xc[1], xc[2], out, 16, 0, true, n,
                          (hipStream_t)stream))
        return PM_EINVAL;
    return launched();
}

}  // extern "C"
